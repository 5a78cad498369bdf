// k_plan_bf16.hip -- the bfloat16 instances of plan_kernel.  This file is
// compiled with the matrix instructions' accumulators and results in VGPRs
// (-mllvm -amdgpu-mfma-vgpr-form): the paired bfloat16 evaluation then keeps
// its activations, the B operands, in AGPRs, and converts each finished
// accumulator pair with one AGPR write instead of two AGPR reads.  The
// binary32 instances stay in k_plan.hip, where that form is slower.
#include "plan_unit.hpp"

namespace voila {

const void* plan_kernel_bf16(int shape) {
    switch (shape) {
#define X(id, ds, na, da, dw, dox, dwz, w, nh) \
    case id:                                   \
        return (const void*)plan_kernel<DT_BF16, ds, na, da, dw, w, nh, plan_mode<w>()>;
        VOILA_SHAPES(X)
#undef X
    }
    return nullptr;
}

}  // namespace voila
