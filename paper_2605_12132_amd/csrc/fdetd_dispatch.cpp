// Host-side dispatch of the row-marching stage kernels on the stencil half width N_D (the kernels are
// compiled per N_D range in separate translation units of fdetd_march.hip).
#include "fdetd_internal.h"

namespace fdetd {

hipError_t launch_maxwell_march(int prec, int nd, const BatchArgs &a, hipStream_t s)
{
    switch (nd) {
#define C_(N) \
    case N: return march_maxwell_nd<N>(prec, a, s);
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14) C_(15) C_(16)
#undef C_
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_envelope_march(int prec, int nd, const BatchArgs &a, hipStream_t s)
{
    switch (nd) {
#define C_(N) \
    case N: return march_envelope_nd<N>(prec, a, s);
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14) C_(15) C_(16)
#undef C_
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stagger_march(int prec, int nd, const BatchArgs &a, hipStream_t s)
{
    switch (nd) {
#define C_(N) \
    case N: return march_stagger_nd<N>(prec, a, s);
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14) C_(15) C_(16)
#undef C_
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_maxwell_any(int prec, const BatchArgs &a, hipStream_t s)
{
    if (a.increment) return hipErrorInvalidValue;  // increment-form plans batch per width
    if (prec == P64) return march_maxwell_any_p64(a, s);
    return a.compensated && a.n == 0 ? march_maxwell_any_p32c(a, s) : march_maxwell_any_p32(a, s);
}

hipError_t launch_stagger_any(int prec, const BatchArgs &a, hipStream_t s)
{
    return prec == P64 ? march_stagger_any_p64(a, s) : march_stagger_any_p32(a, s);
}

// A wavefront of 64 lanes covers 32 z columns in FP64 (a lane pair per complex value) and 64 in FP32 (one
// lane per value); the kernels' lane mapping (elem<double2>::S = 2, elem<float2>::S = 1) matches this.
int march_columns_per_wave(int prec) { return prec == P64 ? 32 : 64; }

}  // namespace fdetd
