// Batched multi-source BFS (placeholder until the batched kernels land).
#include "common.h"

namespace gb {
struct MultiWs {
    void* block = nullptr;
};
void free_multi_ws(MultiWs* w) {
    if (!w) return;
    if (w->block) (void)hipFree(w->block);
    delete w;
}
}  // namespace gb
