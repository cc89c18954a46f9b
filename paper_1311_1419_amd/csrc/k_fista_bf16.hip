// Fused BF16 recovery kernel (placeholder until the fused path lands).
#include "internal.h"
#include "mfma.h"

namespace csv {

void launch_bf16_frag_layout(Operator* op, hipStream_t st) {
    (void)op;
    (void)st;
}

int fused_tile_blocks(int n, int Mp) {
    (void)n;
    (void)Mp;
    return 0;
}

void launch_fista_bf16(const FusedTile*, int, int, int, int, const float*, int*, hipStream_t) {
    throw Error{CSV_EUNSUPPORTED, "BF16 fused recovery is not available in this build"};
}

}  // namespace csv
