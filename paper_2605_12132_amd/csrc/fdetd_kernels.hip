// One-cell-per-thread gfx950 kernels: the operator application used by the plan-time power iteration
// (k_maxwell_apply, k_envelope_apply), current staging, the axis rule, reductions and copies.
//
// Every kernel here is one banded-matrix sweep over a (z, rho) grid (section 2.2): lanes run along z
// (z is the contiguous axis, so a wave's loads of one row are coalesced), the four waves of a workgroup
// cover four consecutive rows, and neighbouring rows' loads are shared through the L1/L2 caches.  The
// time-stepping hot path uses the row-marching kernels of fdetd_march.hip instead.
#include <hip/hip_runtime.h>

#include <climits>

#include "fdetd_internal.h"

namespace fdetd {
namespace {

constexpr int TZ = 64;  // z extent of a workgroup tile (one wave)
constexpr int TR = 4;   // rows per workgroup (one wave each)

template <typename AR>
struct cx {
    AR x, y;
};

template <typename AR>
__device__ __forceinline__ cx<AR> operator+(cx<AR> a, cx<AR> b) { return {a.x + b.x, a.y + b.y}; }
template <typename AR>
__device__ __forceinline__ cx<AR> operator-(cx<AR> a, cx<AR> b) { return {a.x - b.x, a.y - b.y}; }
template <typename AR>
__device__ __forceinline__ cx<AR> operator*(AR s, cx<AR> a) { return {s * a.x, s * a.y}; }
// i * s * a
template <typename AR>
__device__ __forceinline__ cx<AR> times_i(AR s, cx<AR> a) { return {-s * a.y, s * a.x}; }

template <typename V> struct storage;
template <> struct storage<double2> { using R = double; };
template <> struct storage<float2> { using R = float; };

template <typename AR, typename V>
__device__ __forceinline__ cx<AR> ld(const V *p, size_t o)
{
    const V v = p[o];
    return {(AR)v.x, (AR)v.y};
}

// --------------------------------------------------------------------------------------------------
// Maxwell Horner stage: vout = w + coef * H vin (section 2.5 discrete Ampere/Faraday equations).
// Radial values outside the grid follow section 2.4: a primary row q < 0 is row -1-q, a staggered row
// q < 0 is row -q, times the extension sign of the component; rows >= nr and z outside [0, nz) are 0.
// The divergence operands rho*F of D_div^(+-) are formed from the extended F and the signed coordinate
// of the row (negative on the mirror side), which is the extension of rho*F with the opposite sign.
// --------------------------------------------------------------------------------------------------
template <typename AR, typename V, int ND>
__device__ __forceinline__ void maxwell_cell(const MaxwellStageArgs &A, int k, int i, cx<AR> d[6])
{
    const int nz = A.nz, nr = A.nr;
    const size_t P = (size_t)nz * nr;
    const V *vin = (const V *)A.vin;
    const bool addj = A.first && A.has_src;
    const V *jp[3] = {(const V *)A.jr, (const V *)A.jt, (const V *)A.jz};
    const AR beta_in = (AR)A.beta_in;

    auto at = [&](int c, int q, int ii) -> cx<AR> {  // 0 <= q < nr, 0 <= ii < nz
        const size_t o = (size_t)q * nz + ii;
        cx<AR> x = ld<AR>(vin + c * P, o);
        if (addj && c < 3) x = x + beta_in * ld<AR>(jp[c], o);
        return x;
    };
    auto zv = [&](int c, int q, int ii) -> cx<AR> {
        if (ii < 0 || ii >= nz) return {0, 0};
        return at(c, q, ii);
    };
    auto prim = [&](int c, int q, AR par) -> cx<AR> {
        if (q < 0) {
            q = -1 - q;
            if (q >= nr) return {0, 0};
            return par * at(c, q, i);
        }
        if (q >= nr) return {0, 0};
        return at(c, q, i);
    };
    auto stag = [&](int c, int q, AR par, cx<AR> axis) -> cx<AR> {
        if (q == 0) return axis;
        if (q < 0) {
            q = -q;
            if (q >= nr) return {0, 0};
            return par * at(c, q, i);
        }
        if (q >= nr) return {0, 0};
        return at(c, q, i);
    };

    const AR pS = (AR)A.pS, pA = -(AR)A.pS;
    const AR dr = (AR)A.dr;
    const AR mm = (AR)A.m;
    const AR rip = (AR)A.rinv_p[k];
    const AR ris = (AR)A.rinv_s[k];
    const cx<AR> zero = {0, 0};

    // B_z on the axis: extrapolated for m = 0 (constant on the axis), else 0 (section 2.4)
    cx<AR> bz_axis = zero;
    if (A.m == 0 && k < ND) {
#pragma unroll
        for (int q = 1; q <= ND; ++q) bz_axis = bz_axis + (AR)A.cax[q - 1] * at(BZ, q, i);
    }

    // dE_rho = -D_z^(+) B_theta + (i m / rho_(-)) B_z           (staggered rows k >= 1)
    {
        cx<AR> s = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) s = s + (AR)A.az[j - 1] * (zv(BTH, k, i + j) - zv(BTH, k, i - j + 1));
        d[ER] = (k >= 1) ? times_i(mm * ris, at(BZ, k, i)) - s : zero;
    }
    // dE_theta = D_z^(+) B_rho - D_rho^(+,mS) B_z
    {
        cx<AR> s = zero, t = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) {
            s = s + (AR)A.az[j - 1] * (zv(BR, k, i + j) - zv(BR, k, i - j + 1));
            t = t + (AR)A.ar[j - 1] * (stag(BZ, k + j, pS, bz_axis) - stag(BZ, k - j + 1, pS, bz_axis));
        }
        d[ETH] = s - t;
    }
    // dE_z = -(i m / rho) B_rho + rho^-1 D^(+) (rho_(-) B_theta)
    {
        cx<AR> t = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) {
            const int q1 = k + j, q2 = k - j + 1;
            t = t + (AR)A.ar[j - 1] * ((dr * (AR)q1) * stag(BTH, q1, pA, zero) - (dr * (AR)q2) * stag(BTH, q2, pA, zero));
        }
        d[EZ] = rip * t - times_i(mm * rip, at(BR, k, i));
    }
    // dB_rho = D_z^(-) E_theta - (i m / rho) E_z
    {
        cx<AR> s = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) s = s + (AR)A.az[j - 1] * (zv(ETH, k, i + j - 1) - zv(ETH, k, i - j));
        d[BR] = s - times_i(mm * rip, at(EZ, k, i));
    }
    // dB_theta = -D_z^(-) E_rho + D_rho^(-,mS) E_z               (k >= 1)
    {
        cx<AR> s = zero, t = zero;
        if (k >= 1) {
#pragma unroll
            for (int j = 1; j <= ND; ++j) {
                s = s + (AR)A.az[j - 1] * (zv(ER, k, i + j - 1) - zv(ER, k, i - j));
                t = t + (AR)A.ar[j - 1] * (prim(EZ, k + j - 1, pS) - prim(EZ, k - j, pS));
            }
        }
        d[BTH] = t - s;
    }
    // dB_z = (i m / rho_(-)) E_rho - rho_(-)^-1 D^(-) (rho E_theta)  (k >= 1)
    {
        cx<AR> t = zero;
        if (k >= 1) {
#pragma unroll
            for (int j = 1; j <= ND; ++j) {
                const int q1 = k + j - 1, q2 = k - j;
                t = t + (AR)A.ar[j - 1] * ((dr * ((AR)q1 + (AR)0.5)) * prim(ETH, q1, pA) -
                                           (dr * ((AR)q2 + (AR)0.5)) * prim(ETH, q2, pA));
            }
            d[BZ] = times_i(mm * ris, at(ER, k, i)) - ris * t;
        } else {
            d[BZ] = zero;
        }
    }
}

// Error-free sum of two floats (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

template <typename AR, typename V>
__device__ __forceinline__ void maxwell_store(const MaxwellStageArgs &A, int k, int i, const cx<AR> d[6])
{
    const size_t P = (size_t)A.nz * A.nr;
    const size_t o = (size_t)k * A.nz + i;
    const V *psi = (const V *)A.psi;
    V *out = (V *)A.vout;
    const V *jp[3] = {(const V *)A.jr, (const V *)A.jt, (const V *)A.jz};
    const AR coef = (AR)A.coef, beta = (AR)A.beta;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
        const bool axis_slot = (k == 0) && (c == ER || c == BTH || c == BZ);
        // increment relative to psi: beta * Jbar (E slots) + coef * H v
        cx<AR> inc = coef * d[c];
        if (A.has_src && c < 3) inc = inc + beta * ld<AR>(jp[c], o);
        if constexpr (sizeof(V) == 8) {
            if (A.last_compensated) {
                // psi_hi + lo + inc -> (psi_hi, lo), both float, carried exactly by TwoSum
                float2 *lo = (float2 *)A.lo;
                const float2 h = ((const float2 *)psi)[c * P + o];
                const float2 l = lo[c * P + o];
                float sx, ex, sy, ey;
                two_sum(h.x, (float)(inc.x + (AR)l.x), sx, ex);
                two_sum(h.y, (float)(inc.y + (AR)l.y), sy, ey);
                if (axis_slot) sx = sy = ex = ey = 0.f;
                out[c * P + o] = V{sx, sy};
                lo[c * P + o] = float2{ex, ey};
                continue;
            }
        }
        cx<AR> w = ld<AR>(psi + c * P, o) + inc;
        if (axis_slot) w = {0, 0};
        out[c * P + o] = V{(typename storage<V>::R)w.x, (typename storage<V>::R)w.y};
    }
}

template <typename V, int ND>
__global__ __launch_bounds__(TZ *TR) void k_maxwell_apply(MaxwellStageArgs A)
{
    using R = typename storage<V>::R;
    const int i = blockIdx.x * TZ + threadIdx.x;
    const int k = blockIdx.y * TR + threadIdx.y;
    if (i >= A.nz || k >= A.nr) return;
    if constexpr (sizeof(R) == 4) {
        if (k < A.axis_rows) {  // near-axis rows: 1/rho amplifies rounding, keep FP64 arithmetic
            cx<double> d[6];
            maxwell_cell<double, V, ND>(A, k, i, d);
            maxwell_store<double, V>(A, k, i, d);
            return;
        }
    }
    cx<R> d[6];
    maxwell_cell<R, V, ND>(A, k, i, d);
    maxwell_store<R, V>(A, k, i, d);
}

// --------------------------------------------------------------------------------------------------
// Envelope Horner stage (section 4.2):  out = psi + coef * H_a vin,
//   H_a (a, a~) = (a~, (L_rho + L_z - m^2/rho^2 - chi) a + 2 i k0 (D_z^(C) a + a~)),
// L_rho = D^2 + rho^-1 D^(C) with the scalar-like (mS) extension at rho < 0.
// --------------------------------------------------------------------------------------------------
template <typename AR, typename V, int ND>
__device__ __forceinline__ void envelope_cell(const EnvelopeStageArgs &A, int k, int i)
{
    using R = typename storage<V>::R;
    const int nz = A.nz, nr = A.nr;
    const V *va = (const V *)A.vin_a;
    const size_t o = (size_t)k * nz + i;
    const AR pS = (AR)A.pS;
    auto rv = [&](int q) -> cx<AR> {
        if (q < 0) {
            q = -1 - q;
            if (q >= nr) return {0, 0};
            return pS * ld<AR>(va, (size_t)q * nz + i);
        }
        if (q >= nr) return {0, 0};
        return ld<AR>(va, (size_t)q * nz + i);
    };
    auto zv = [&](int ii) -> cx<AR> {
        if (ii < 0 || ii >= nz) return {0, 0};
        return ld<AR>(va, (size_t)k * nz + ii);
    };
    const cx<AR> a0 = ld<AR>(va, o);
    cx<AR> lr = (AR)A.br[0] * a0, dr1 = {0, 0}, lz = (AR)A.bz[0] * a0, dz1 = {0, 0};
#pragma unroll
    for (int j = 1; j <= ND; ++j) {
        const cx<AR> rp = rv(k + j), rm = rv(k - j);
        lr = lr + (AR)A.br[j] * (rp + rm);
        dr1 = dr1 + (AR)A.drc[j - 1] * (rp - rm);
        const cx<AR> zp = zv(i + j), zm = zv(i - j);
        lz = lz + (AR)A.bz[j] * (zp + zm);
        dz1 = dz1 + (AR)A.dzc[j - 1] * (zp - zm);
    }
    const cx<AR> tin = ld<AR>((const V *)A.vin_t, o);
    const AR pot = (AR)A.m2rinv2[k] + (AR)((const R *)A.chi)[o];
    const cx<AR> da = tin;
    const cx<AR> dt = lr + (AR)A.rinv_p[k] * dr1 + lz - pot * a0 + times_i((AR)(2.0 * A.k0), dz1 + tin);
    const AR coef = (AR)A.coef;
    const cx<AR> ia = coef * da, it = coef * dt;
    if constexpr (sizeof(R) == 4) {
        if (A.last_compensated) {
            float2 *loa = (float2 *)A.lo_a, *lot = (float2 *)A.lo_t;
            const float2 ha = ((const float2 *)A.psi_a)[o], ht = ((const float2 *)A.psi_t)[o];
            const float2 la = loa[o], lt = lot[o];
            float s0, e0, s1, e1, s2, e2, s3, e3;
            two_sum(ha.x, (float)(ia.x + (AR)la.x), s0, e0);
            two_sum(ha.y, (float)(ia.y + (AR)la.y), s1, e1);
            two_sum(ht.x, (float)(it.x + (AR)lt.x), s2, e2);
            two_sum(ht.y, (float)(it.y + (AR)lt.y), s3, e3);
            ((float2 *)A.out_a)[o] = float2{s0, s1};
            ((float2 *)A.out_t)[o] = float2{s2, s3};
            loa[o] = float2{e0, e1};
            lot[o] = float2{e2, e3};
            return;
        }
    }
    const cx<AR> wa = ld<AR>((const V *)A.psi_a, o) + ia;
    const cx<AR> wt = ld<AR>((const V *)A.psi_t, o) + it;
    ((V *)A.out_a)[o] = V{(R)wa.x, (R)wa.y};
    ((V *)A.out_t)[o] = V{(R)wt.x, (R)wt.y};
}

template <typename V, int ND>
__global__ __launch_bounds__(TZ *TR) void k_envelope_apply(EnvelopeStageArgs A)
{
    using R = typename storage<V>::R;
    const int i = blockIdx.x * TZ + threadIdx.x;
    const int k = blockIdx.y * TR + threadIdx.y;
    if (i >= A.nz || k >= A.nr) return;
    if constexpr (sizeof(R) == 4) {
        if (k < A.axis_rows) {
            envelope_cell<double, V, ND>(A, k, i);
            return;
        }
    }
    envelope_cell<R, V, ND>(A, k, i);
}

// --------------------------------------------------------------------------------------------------
// rho = 0 slots of E_rho, B_theta, B_z after a step (section 2.4): constant components take the
// extrapolation sum c_k' F_k' (B_z for m = 0, E_rho and B_theta for m = 1); all others are 0.
// --------------------------------------------------------------------------------------------------
template <typename V, int ND>
__global__ __launch_bounds__(256) void k_axis_fix(AxisArgs A)
{
    using R = typename storage<V>::R;
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= A.nz) return;
    const size_t P = (size_t)A.nz * A.nr;
    V *psi = (V *)A.psi;
    const int comps[3] = {ER, BTH, BZ};
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int c = comps[t];
        const bool extrap = (c == BZ) ? (A.m == 0) : (A.m == 1);
        cx<double> s = {0, 0};
        if (extrap) {
#pragma unroll
            for (int q = 1; q <= ND; ++q) s = s + A.cax[q - 1] * ld<double>(psi + c * P, (size_t)q * A.nz + i);
        }
        psi[c * P + i] = V{(R)s.x, (R)s.y};
    }
}

// The axis rule for every problem of a batch: grid.y = problem, threads over the columns; the weights and
// N_D come from the problem's descriptor, the sum runs in the order of k_axis_fix (same results).
template <typename V>
__global__ __launch_bounds__(256) void k_axis_fix_batch(BatchArgs A)
{
    using R = typename storage<V>::R;
    const ProbDesc &D = A.probs[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= D.nz) return;
    const size_t P = D.plane;
    V *psi = (V *)A.psi[blockIdx.y];
    const int comps[3] = {ER, BTH, BZ};
#pragma unroll
    for (int t = 0; t < 3; ++t) {
        const int c = comps[t];
        const bool extrap = (c == BZ) ? (D.m == 0) : (D.m == 1);
        cx<double> s = {0, 0};
        if (extrap)
            for (int q = 1; q <= D.nd; ++q) s = s + D.cax[q - 1] * ld<double>(psi + c * P, (size_t)q * D.nz + i);
        psi[c * P + i] = V{(R)s.x, (R)s.y};
    }
}

// --------------------------------------------------------------------------------------------------
// Reductions for the plan-time power iteration: per-block sums of |x|^2 (wave shuffles, then LDS).
// --------------------------------------------------------------------------------------------------
template <typename V>
__global__ __launch_bounds__(256) void k_norm2(const V *x, size_t n, double *partial)
{
    double acc = 0.0;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
        const V v = x[q];
        acc += (double)v.x * v.x + (double)v.y * v.y;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    __shared__ double wsum[4];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

template <typename V>
__global__ __launch_bounds__(256) void k_scale(V *x, size_t n, double alpha)
{
    using R = typename storage<V>::R;
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
        V v = x[q];
        x[q] = V{(R)(alpha * v.x), (R)(alpha * v.y)};
    }
}

__global__ __launch_bounds__(256) void k_copy8(const uint2 *src, uint2 *dst, size_t n)
{
    for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) dst[q] = src[q];
}

// SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the generator's output function applied to a counter.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
constexpr unsigned long long kSplitMixGamma = 0x9E3779B97F4A7C15ull;

// Current blocks of one step of the captured time loop (see JgenArgs): each block strides over the cells
// of every problem in turn, each cell's three components written at once.
template <typename V>
__global__ __launch_bounds__(256) void k_jgen(JgenArgs A)
{
    using R = typename storage<V>::R;
    const double t = (A.step + 0.5);
    for (int p = 0; p < A.nprob; ++p) {
        const ProbDesc &D = A.probs[p];
        const size_t n = D.plane;
        V *j = (V *)A.j[p];
        unsigned long long h = splitmix64(A.seed + kSplitMixGamma);
        h = splitmix64(h + (unsigned long long)(A.step + 1) * kSplitMixGamma);
        h = splitmix64(h + (unsigned long long)(A.pidx[p] + 1) * kSplitMixGamma);
        const double tb = t * D.dt, zb = A.z0f * D.nz * D.dz + A.vb * tb;
        for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
            const int k = (int)(q / D.nz), i = (int)(q % D.nz);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                double re = 0.0, im = 0.0;
                if (A.mode == 1) {
                    const unsigned long long v = (((unsigned long long)c * D.nr + k) * D.nz + i) * 2;
                    const unsigned long long ur = splitmix64(h + (v + 1) * kSplitMixGamma);
                    const unsigned long long ui = splitmix64(h + (v + 2) * kSplitMixGamma);
                    re = ((double)(ur >> 11) * 0x1p-53 * 2.0 - 1.0) * A.amp;
                    im = D.m == 0 ? 0.0 : ((double)(ui >> 11) * 0x1p-53 * 2.0 - 1.0) * A.amp;
                    if (c == 2 && D.m == 0) {
                        const double zs = (i - 0.5) * D.dz, rp = (k + 0.5) * D.dr;
                        re += -A.nb * exp(-((zs - zb) * (zs - zb)) / (2 * A.sigz * A.sigz) - rp * rp / (2 * A.sigr * A.sigr));
                    }
                }
                j[c * n + q] = V{(R)re, (R)im};
            }
        }
    }
}

// E part of w_N = psi + beta_in Jbar (the argument of the highest power of H in the Horner form of the
// midpoint solution of section 2.1) for every problem of a batch, into the E planes of the problem's
// second stage buffer: the input of the B half of a step's first Horner stage where that stage does not
// form it itself (increment form, FP32C at N = 1, FDETD_PLAN_SEPARATE_WN).  Jbar_rho is the staged
// plane, J_theta the corrected one when the plan corrects the current, J_z the caller's.  FP64 arithmetic,
// one rounding to the storage precision.  Each block strides over the cells of every problem in turn.
template <typename V>
__global__ __launch_bounds__(256) void k_form_wn(BatchArgs A)
{
    using R = typename storage<V>::R;
    for (int p = 0; p < A.nprob; ++p) {
        const ProbDesc &D = A.probs[p];
        const size_t n = D.plane;
        const V *psi = (const V *)A.psi[p];
        const V *jc = (const V *)A.aux[p];
        const V *src[3] = {(const V *)D.jbar, D.jth ? (const V *)D.jth : jc + n, jc + 2 * n};
        V *w = (V *)D.buf[1];
        for (size_t q = (size_t)blockIdx.x * 256 + threadIdx.x; q < n; q += (size_t)gridDim.x * 256) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const V x = A.increment ? V{0, 0} : psi[c * n + q], j = src[c][q];
                w[c * n + q] = V{(R)__builtin_fma(A.beta_in, (double)j.x, (double)x.x),
                                 (R)__builtin_fma(A.beta_in, (double)j.y, (double)x.y)};
            }
        }
    }
}

// compile-time dispatch over the stencil half width N_D = 1..16
template <template <typename, int> class L, typename V, typename Args>
hipError_t dispatch_nd(int nd, const Args &a, dim3 grid, dim3 block, hipStream_t s)
{
    switch (nd) {
#define FDETD_CASE(N) \
    case N: return L<V, N>::go(a, grid, block, s);
        FDETD_CASE(1) FDETD_CASE(2) FDETD_CASE(3) FDETD_CASE(4) FDETD_CASE(5) FDETD_CASE(6) FDETD_CASE(7)
        FDETD_CASE(8) FDETD_CASE(9) FDETD_CASE(10) FDETD_CASE(11) FDETD_CASE(12) FDETD_CASE(13)
        FDETD_CASE(14) FDETD_CASE(15) FDETD_CASE(16)
#undef FDETD_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename V, int ND>
struct MaxwellL {
    static hipError_t go(const MaxwellStageArgs &a, dim3 g, dim3 b, hipStream_t s)
    {
        hipLaunchKernelGGL((k_maxwell_apply<V, ND>), g, b, 0, s, a);
        return hipGetLastError();
    }
};
template <typename V, int ND>
struct EnvelopeL {
    static hipError_t go(const EnvelopeStageArgs &a, dim3 g, dim3 b, hipStream_t s)
    {
        hipLaunchKernelGGL((k_envelope_apply<V, ND>), g, b, 0, s, a);
        return hipGetLastError();
    }
};
template <typename V, int ND>
struct AxisL {
    static hipError_t go(const AxisArgs &a, dim3 g, dim3 b, hipStream_t s)
    {
        hipLaunchKernelGGL((k_axis_fix<V, ND>), g, b, 0, s, a);
        return hipGetLastError();
    }
};

dim3 tile_grid(int nz, int nr) { return dim3((nz + TZ - 1) / TZ, (nr + TR - 1) / TR, 1); }

// --------------------------------------------------------------------------------------------------
// Deposition of point samples moving with vz along z (sections 3.2, 3.5, 3.6): J_z(i - 1/2, k) of mode m
// gains q w (F_-(i) - F_+(i)) / dt * R_k * A_m, where F_-+ are the cubic-spline weights left of i - 1/2 of
// the positions z -+ vz dt/2 (the integrated shape, with the sign of the discrete continuity equation),
// R_k the radial shape (rho_k^(eps-1) times the spline weight, the part beyond the axis folded back with
// fold_mS: the m_S type (-1)^m for m <= 1, antisymmetric for m > 1; normalised by sum_k h_k rho_k^eps (even
// fold of the weight) dr with h_0 = 7/8, h_1 = 73/72)
// and A_m the angular shape: 1/(2 pi) for m = 0, e^(-i m theta)/pi otherwise.  A sample whose z shape
// reaches past a z end is not deposited.  One thread per sample; shapes in FP64; atomic adds.
// --------------------------------------------------------------------------------------------------
__device__ __forceinline__ double bspline3(double x)
{
    x = fabs(x);
    if (x < 1.0) return 2.0 / 3.0 - x * x + 0.5 * x * x * x;
    if (x < 2.0) {
        const double t = 2.0 - x;
        return t * t * t / 6.0;
    }
    return 0.0;
}

// rho_k^e; the exponents the radial shape meets for eps in {0, 1/2, 1} by their exact operations (one
// division or square root instead of a pow)
__device__ __forceinline__ double rk_pow(double rk, double e)
{
    if (e == 0.0) return 1.0;
    if (e == 1.0) return rk;
    if (e == -1.0) return 1.0 / rk;
    if (e == 0.5) return sqrt(rk);
    if (e == -0.5) return 1.0 / sqrt(rk);
    return pow(rk, e);
}

// Sign with which the part of a sample's radial shape below the axis is folded back (section 3.5): the
// component's m_S or m_A type for m = 0, 1, antisymmetric for every m > 1 (a sample on the axis then
// deposits nothing into those modes).
__device__ __forceinline__ double fold_mS(int m) { return m > 1 ? -1.0 : (m % 2 == 0 ? 1.0 : -1.0); }
__device__ __forceinline__ double fold_mA(int m) { return m > 1 ? -1.0 : (m == 1 ? 1.0 : -1.0); }

// Radial shape of a sample at rho on the primary rows k = kc - 3 + j, j = 0..6 (folded with parity par,
// normalised by N; w[j] = 0 off [k0, k1]) and the angular shape of mode m at the sample's angle theta,
// given by (x, y): e^(-i m theta) as the m-th power of (x - i y) / rho (theta = 0 on the axis).  Each
// row's spline values and power of rho_k are formed once, for N and the weight.
struct SampleShape {
    int kc, k0, k1;  // rows kc - 3 .. kc + 3, clipped to [0, nr)
    double ar, ai;
    double w[7];
};
__device__ __forceinline__ SampleShape sample_shape(const ProbDesc &D, double rho, double x, double y, double eps,
                                                    double par)
{
    SampleShape S;
    const double dr = D.dr;
    S.kc = (int)floor(rho / dr);
    S.k0 = S.kc - 3 > 0 ? S.kc - 3 : 0;
    S.k1 = S.kc + 3 < D.nr - 1 ? S.kc + 3 : D.nr - 1;
    double N = 0.0;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int k = S.kc - 3 + j;
        S.w[j] = 0.0;
        if (k < 0) continue;  // N sums rows k0 .. kc + 3, beyond the last row too
        const double rk = (k + 0.5) * dr;
        const double bp = bspline3((rk - rho) / dr), bm = bspline3((-rk - rho) / dr);
        const double t = rk_pow(rk, eps - 1.0);
        N += (k == 0 ? 7.0 / 8.0 : (k == 1 ? 73.0 / 72.0 : 1.0)) * (rk * t) * (bp + bm) * dr;
        if (k <= S.k1) S.w[j] = t * (bp + par * bm);
    }
    const double inv = 1.0 / N;
#pragma unroll
    for (int j = 0; j < 7; ++j) S.w[j] *= inv;
    if (D.m == 0) {
        S.ar = 0.5 / M_PI;
        S.ai = 0.0;
    } else {
        const double c1 = rho > 0.0 ? x / rho : 1.0, s1 = rho > 0.0 ? y / rho : 0.0;
        double cr = 1.0, ci = 0.0;  // cos, sin of m theta
        for (int j = 0; j < D.m; ++j) {
            const double t = cr * c1 - ci * s1;
            ci = cr * s1 + ci * c1;
            cr = t;
        }
        S.ar = cr / M_PI;
        S.ai = -ci / M_PI;
    }
    return S;
}
// The z shape of a position x (in cells) spans nodes floor(x) - 1 .. floor(x) + 2, which must lie on the grid.
__device__ __forceinline__ bool z_on_grid(const ProbDesc &D, double x)
{
    return (int)floor(x) - 1 >= 0 && (int)floor(x) + 2 <= D.nz - 1;
}

// Block-wide min and max of four ints (NW wave64 wavefronts), through LDS (red holds 4 NW ints).
template <int NW = 4>
__device__ __forceinline__ void block_minmax(int v[4], int *red)
{
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int x = v[c];
        for (int o = 32; o > 0; o >>= 1) {
            const int y = __shfl_xor(x, o);
            x = (c & 1) ? max(x, y) : min(x, y);  // c = 0, 2: min; 1, 3: max
        }
        if (lane == 0) red[4 * wv + c] = x;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        int x = red[c];
        for (int w = 1; w < NW; ++w) x = (c & 1) ? max(x, red[4 * w + c]) : min(x, red[4 * w + c]);
        v[c] = x;
    }
    __syncthreads();
}

// J_z (plane jz) and, when rxy is not null, the planar density differential of one sample whose
// integrated z shape spans more than 8 nodes (it moves more than 3 cells in a step): the nodes lo .. hi
// one by one, F_-+ summed on the way, every add a global atomic.  The radial and angular factors of the
// two half-step positions are Sp, Sm (the same shape twice for a sample moving along z only), averaged
// for J_z and differenced for rho_xy, as in the narrow path.
template <typename R>
__device__ void deposit_z_wide(R *jz, R *rxy, const ProbDesc &D, const SampleShape &Sp, const SampleShape &Sm,
                               double qw, double zp, double zm, int lo, int hi, double inv_dt, double inv_dz)
{
    const int k0 = min(Sp.k0, Sm.k0), k1 = max(Sp.k1, Sm.k1);
    double Fp = 0.0, Fm = 0.0;
    for (int i = lo; i <= hi; ++i) {
        const double dF = (Fm - Fp) * inv_dt;
        const double bp = bspline3(i - zp), bm = bspline3(i - zm);
        Fp += bp;
        Fm += bm;
        const double sz = 0.5 * (bp + bm) * inv_dz;
        if (dF == 0.0 && (rxy == nullptr || sz == 0.0)) continue;
        for (int k = k0; k <= k1; ++k) {
            const int jp = k - Sp.kc + 3, jm = k - Sm.kc + 3;
            const double wp = (jp >= 0 && jp < 7) ? Sp.w[jp] : 0.0, wm = (jm >= 0 && jm < 7) ? Sm.w[jm] : 0.0;
            if (wp == 0.0 && wm == 0.0) continue;
            const size_t o = 2 * ((size_t)k * D.nz + i);
            if (dF != 0.0) {
                atomicAdd(jz + o, (R)(qw * dF * 0.5 * (wp * Sp.ar + wm * Sm.ar)));
                atomicAdd(jz + o + 1, (R)(qw * dF * 0.5 * (wp * Sp.ai + wm * Sm.ai)));
            }
            if (rxy != nullptr && sz != 0.0) {
                atomicAdd(rxy + o, (R)(qw * sz * (wp * Sp.ar - wm * Sm.ar) * inv_dt));
                atomicAdd(rxy + o + 1, (R)(qw * sz * (wp * Sp.ai - wm * Sm.ai) * inv_dt));
            }
        }
    }
}

// J_z of the samples of a block (DEP_PER_THREAD per thread, consecutive).  For each problem the block
// forms the footprint of its samples (the nodes and rows their shapes touch); when it fits an LDS tile of
// DEP_TILE cells -- samples given in position order, as PIC codes keep them, make the footprint of a block
// small -- the adds go to the tile (FP64 LDS atomics) and the tile is added to the grid once, one global
// atomic per touched cell; otherwise every add is a global atomic.  Either way the result is the same sum.
constexpr int DEP_PER_THREAD = 4, DEP_TILE = 4096;
template <typename R>
__global__ __launch_bounds__(256) void k_deposit_jz(DepositArgs A)
{
    __shared__ double tile[2 * DEP_TILE];
    __shared__ int red[16];
    const int64_t s0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * DEP_PER_THREAD;
    struct Smp { double z, rho, x, y, qw; bool ok; };
    Smp sm[DEP_PER_THREAD];
#pragma unroll
    for (int u = 0; u < DEP_PER_THREAD; ++u) {
        const int64_t s = s0 + u;
        sm[u].ok = s < A.n;
        const int64_t sc = sm[u].ok ? s : 0;
        const double x = A.samples[4 * sc + 1], y = A.samples[4 * sc + 2];
        sm[u].z = A.samples[4 * sc] + A.shift;  // samples moved along z (0 for fdetd_deposit_jz)
        sm[u].qw = A.samples[4 * sc + 3];
        sm[u].rho = sqrt(x * x + y * y);
        sm[u].x = x;
        sm[u].y = y;
    }
    for (int p = 0; p < A.nprob; ++p) {
        const ProbDesc &D = A.probs[p];
        // footprints: nodes lo .. hi, rows kc - 3 .. kc + 3 (clipped)
        int lo[DEP_PER_THREAD], hi[DEP_PER_THREAD];
        bool wide[DEP_PER_THREAD];
        int fp[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};  // zmin, zmax, kmin, kmax
#pragma unroll
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            const double zp = (sm[u].z + 0.5 * A.vz * D.dt) / D.dz, zm = (sm[u].z - 0.5 * A.vz * D.dt) / D.dz;
            lo[u] = (int)floor(fmin(zp, zm)) - 1;
            hi[u] = (int)floor(fmax(zp, zm)) + 2;
            wide[u] = false;
            if (!sm[u].ok || !z_on_grid(D, zp) || !z_on_grid(D, zm)) {
                hi[u] = lo[u] - 1;  // nothing to deposit
                continue;
            }
            // more than 8 nodes: deposited by deposit_z_wide, outside the block's tile
            wide[u] = hi[u] - lo[u] + 1 > 8;
            if (wide[u]) continue;
            const int kc = (int)floor(sm[u].rho / D.dr);
            fp[0] = min(fp[0], lo[u]);
            fp[1] = max(fp[1], hi[u]);
            fp[2] = min(fp[2], max(kc - 3, 0));
            fp[3] = max(fp[3], min(kc + 3, D.nr - 1));
        }
        block_minmax(fp, red);
        // fp covers the narrow samples only; without any the tile is empty (wide samples add directly)
        const int tz = fp[1] >= fp[0] ? fp[1] - fp[0] + 1 : 0, tr = fp[1] >= fp[0] ? fp[3] - fp[2] + 1 : 0;
        const bool use_tile = tz > 0 && (int64_t)tz * tr <= DEP_TILE;  // uniform across the block
        R *jz = (R *)A.j[p] + 2 * 2 * D.plane;               // plane 2, interleaved complex
        const double inv_dt = 1.0 / D.dt, par_s = fold_mS(D.m);
        if (use_tile) {
            for (int c = threadIdx.x; c < 2 * tz * tr; c += 256) tile[c] = 0.0;
            __syncthreads();
        }
#pragma unroll
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            if (hi[u] < lo[u]) continue;
            const double zp = (sm[u].z + 0.5 * A.vz * D.dt) / D.dz, zm = (sm[u].z - 0.5 * A.vz * D.dt) / D.dz;
            if (wide[u]) {
                const SampleShape S = sample_shape(D, sm[u].rho, sm[u].x, sm[u].y, A.eps, par_s);
                deposit_z_wide<R>(jz, nullptr, D, S, S, sm[u].qw, zp, zm, lo[u], hi[u], inv_dt, 1.0 / D.dz);
                continue;
            }
            double dF[8];
            double Fp = 0.0, Fm = 0.0;
            for (int v = 0; v <= hi[u] - lo[u]; ++v) {
                dF[v] = (Fm - Fp) * inv_dt;
                Fp += bspline3(lo[u] + v - zp);
                Fm += bspline3(lo[u] + v - zm);
            }
            const SampleShape S = sample_shape(D, sm[u].rho, sm[u].x, sm[u].y, A.eps, par_s);
#pragma unroll
            for (int jr = 0; jr < 7; ++jr) {
                const int k = S.kc - 3 + jr;
                const double rs = S.w[jr];
                if (rs == 0.0) continue;
                for (int v = 0; v <= hi[u] - lo[u]; ++v) {
                    const double w = sm[u].qw * dF[v] * rs;
                    if (w == 0.0) continue;
                    if (use_tile) {
                        double *c = tile + 2 * ((k - fp[2]) * tz + lo[u] + v - fp[0]);
                        atomicAdd(c, w * S.ar);
                        atomicAdd(c + 1, w * S.ai);
                    } else {
                        R *c = jz + 2 * ((size_t)k * D.nz + lo[u] + v);
                        atomicAdd(c, (R)(w * S.ar));
                        atomicAdd(c + 1, (R)(w * S.ai));
                    }
                }
            }
        }
        if (use_tile) {
            __syncthreads();
            for (int c = threadIdx.x; c < tz * tr; c += 256) {
                const double re = tile[2 * c], im = tile[2 * c + 1];
                if (re == 0.0 && im == 0.0) continue;
                R *g = jz + 2 * ((size_t)(fp[2] + c / tz) * D.nz + fp[0] + c % tz);
                atomicAdd(g, (R)re);
                atomicAdd(g + 1, (R)im);
            }
            __syncthreads();  // the tile is reused by the next problem
        }
    }
}

// Currents of moving samples (section 3.6) and the planar density differential (section 3.7), one thread
// per sample (z, x, y, q w, v_x, v_y, v_z, unused), positions +- v dt/2:
//   J_rho, J_theta += q w v_rho|theta S(z_p) R_A(rho_p) A(theta_p)          (planes 0, 1)
//   J_z(i - 1/2)   += q w dF(i) (R_S(rho+) A(theta+) + R_S(rho-) A(theta-)) / 2  (plane 2)
//   rho_xy         += q w (S(z+) + S(z-)) / 2 (R_S(rho+) A(theta+) - R_S(rho-) A(theta-)) / dt  (plane 3)
// R_A / R_S: radial shape folded with fold_mA / fold_mS.  Samples whose z shapes leave the grid are
// skipped.
// As k_deposit_jz, blocks of DEP_PER_THREAD x 256 consecutive samples accumulate in an LDS tile of
// DEP_TILE_CUR cells (all planes) when their footprint fits.  A sample whose integrated z shape spans more
// than 8 nodes (it moves more than 3 cells in a step) adds everything with global atomics instead.
constexpr int DEP_TILE_CUR = 1024;
template <typename R>
__global__ __launch_bounds__(256) void k_deposit_current(DepositArgs A)
{
    __shared__ double tile[2 * 4 * DEP_TILE_CUR];
    __shared__ int red[16];
    const int64_t s0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * DEP_PER_THREAD;
    const int npl = A.rho_xy ? 4 : 3;
    for (int p = 0; p < A.nprob; ++p) {
        const ProbDesc &D = A.probs[p];
        const double h = 0.5 * D.dt;
        auto sample = [&](int u) { const int64_t s = s0 + u; return A.samples + 8 * (s < A.n ? s : 0); };
        auto on_grid = [&](int u, double &zp, double &zm) {
            const double *q = sample(u);
            zp = (q[0] + h * q[6]) / D.dz;
            zm = (q[0] - h * q[6]) / D.dz;
            return s0 + u < A.n && z_on_grid(D, zp) && z_on_grid(D, zm);
        };
        auto is_wide = [&](double zp, double zm) {
            return (int)floor(fmax(zp, zm)) + 2 - ((int)floor(fmin(zp, zm)) - 1) + 1 > 8;
        };
        auto rows_of = [&](double r, int &k0, int &k1) {
            const int kc = (int)floor(r / D.dr);
            k0 = kc - 3 > 0 ? kc - 3 : 0;
            k1 = kc + 3 < D.nr - 1 ? kc + 3 : D.nr - 1;
        };
        int fp[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};  // zmin, zmax, kmin, kmax
#pragma unroll
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            double zp, zm;
            if (!on_grid(u, zp, zm) || is_wide(zp, zm)) continue;
            const double *q = sample(u);
            fp[0] = min(fp[0], (int)floor(fmin(zp, zm)) - 1);
            fp[1] = max(fp[1], (int)floor(fmax(zp, zm)) + 2);
            const double xs[3] = {q[1], q[1] + h * q[4], q[1] - h * q[4]}, ys[3] = {q[2], q[2] + h * q[5], q[2] - h * q[5]};
            for (int c = 0; c < 3; ++c) {
                int a, b;
                rows_of(sqrt(xs[c] * xs[c] + ys[c] * ys[c]), a, b);
                fp[2] = min(fp[2], a);
                fp[3] = max(fp[3], b);
            }
        }
        block_minmax(fp, red);
        // fp covers the narrow samples only; without any the tile is empty (wide samples add directly)
        const int tz = fp[1] >= fp[0] ? fp[1] - fp[0] + 1 : 0, tr = fp[1] >= fp[0] ? fp[3] - fp[2] + 1 : 0;
        const bool use_tile = tz > 0 && (int64_t)tz * tr <= DEP_TILE_CUR;  // uniform across the block
        R *j = (R *)A.j[p];
        const size_t pl = 2 * D.plane;  // one plane in R units (interleaved complex)
        if (use_tile) {
            for (int c = threadIdx.x; c < 2 * npl * tz * tr; c += 256) tile[c] = 0.0;
            __syncthreads();
        }
        const double inv_dt = 1.0 / D.dt, inv_dz = 1.0 / D.dz;
        const double par_s = fold_mS(D.m), par_a = fold_mA(D.m);
        bool tiled = use_tile;  // false for a wide sample
        auto add = [&](int plane, int k, int i, double re, double im) {
            if (tiled) {
                double *c = tile + 2 * ((plane * tr + k - fp[2]) * tz + i - fp[0]);
                atomicAdd(c, re);
                atomicAdd(c + 1, im);
            } else {
                R *c = j + plane * pl + 2 * ((size_t)k * D.nz + i);
                atomicAdd(c, (R)re);
                atomicAdd(c + 1, (R)im);
            }
        };
#pragma unroll 1
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            double zp, zm;
            if (!on_grid(u, zp, zm)) continue;
            const bool wide = is_wide(zp, zm);
            tiled = use_tile && !wide;
            const double *q = sample(u);
            const double z = q[0], x = q[1], y = q[2], qw = q[3], vx = q[4], vy = q[5];
            const double r0 = sqrt(x * x + y * y), zc = z / D.dz;
            const double vr = r0 > 0.0 ? (x * vx + y * vy) / r0 : 0.0, vt = r0 > 0.0 ? (x * vy - y * vx) / r0 : 0.0;
            const double xp = x + h * vx, yp = y + h * vy, xm = x - h * vx, ym = y - h * vy;
            const double rp = sqrt(xp * xp + yp * yp), rm = sqrt(xm * xm + ym * ym);
            // transverse currents at the sample (m_A fold)
            if (vr != 0.0 || vt != 0.0) {
                const SampleShape S0 = sample_shape(D, r0, x, y, A.eps, par_a);
                const int lo = (int)floor(zc) - 1;
                double wz[4];
#pragma unroll
                for (int u2 = 0; u2 < 4; ++u2) wz[u2] = qw * bspline3(lo + u2 - zc) * inv_dz;
#pragma unroll
                for (int jr = 0; jr < 7; ++jr) {
                    const int k = S0.kc - 3 + jr;
                    const double rs = S0.w[jr];
                    if (rs == 0.0) continue;
                    for (int u2 = 0; u2 < 4; ++u2) {
                        const double w = wz[u2] * rs;
                        if (w == 0.0) continue;
                        add(0, k, lo + u2, w * vr * S0.ar, w * vr * S0.ai);
                        add(1, k, lo + u2, w * vt * S0.ar, w * vt * S0.ai);
                    }
                }
            }
            // longitudinal current and planar density differential over the nodes of both z shapes
            const int lo = (int)floor(fmin(zp, zm)) - 1, hi = (int)floor(fmax(zp, zm)) + 2;
            if (wide) {
                const SampleShape Sp = sample_shape(D, rp, xp, yp, A.eps, par_s), Sm = sample_shape(D, rm, xm, ym, A.eps, par_s);
                deposit_z_wide<R>(j + 2 * pl, A.rho_xy ? j + 3 * pl : nullptr, D, Sp, Sm, qw, zp, zm, lo, hi, inv_dt, inv_dz);
                continue;
            }
            double dF[8], sz[8];  // nodes lo .. hi (at most 8), 0 beyond
            double Fp = 0.0, Fm = 0.0;
#pragma unroll
            for (int v = 0; v < 8; ++v) {
                dF[v] = sz[v] = 0.0;
                if (v > hi - lo) continue;
                dF[v] = (Fm - Fp) * inv_dt;
                const double bp = bspline3(lo + v - zp), bm = bspline3(lo + v - zm);
                Fp += bp;
                Fm += bm;
                sz[v] = 0.5 * (bp + bm) * inv_dz;
            }
            // rows of both shapes
            const SampleShape Sp = sample_shape(D, rp, xp, yp, A.eps, par_s), Sm = sample_shape(D, rm, xm, ym, A.eps, par_s);
            const int k0 = min(Sp.k0, Sm.k0), k1 = max(Sp.k1, Sm.k1);
            for (int k = k0; k <= k1; ++k) {
                const int jp = k - Sp.kc + 3, jm = k - Sm.kc + 3;
                double wp = 0.0, wm = 0.0;  // selects with static indices keep the shapes in registers
#pragma unroll
                for (int q = 0; q < 7; ++q) {
                    wp = jp == q ? Sp.w[q] : wp;
                    wm = jm == q ? Sm.w[q] : wm;
                }
                if (wp == 0.0 && wm == 0.0) continue;
                const double sr = 0.5 * (wp * Sp.ar + wm * Sm.ar), si = 0.5 * (wp * Sp.ai + wm * Sm.ai);
                const double dr_ = (wp * Sp.ar - wm * Sm.ar) * inv_dt, di = (wp * Sp.ai - wm * Sm.ai) * inv_dt;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    if (dF[v] != 0.0) add(2, k, lo + v, qw * dF[v] * sr, qw * dF[v] * si);
                    if (A.rho_xy && sz[v] != 0.0) add(3, k, lo + v, qw * sz[v] * dr_, qw * sz[v] * di);
                }
            }
        }
        if (use_tile) {
            __syncthreads();
            for (int c = threadIdx.x; c < npl * tz * tr; c += 256) {
                const double re = tile[2 * c], im = tile[2 * c + 1];
                if (re == 0.0 && im == 0.0) continue;
                const int plane = c / (tz * tr), cell = c % (tz * tr);
                R *g = j + plane * pl + 2 * ((size_t)(fp[2] + cell / tz) * D.nz + fp[0] + cell % tz);
                atomicAdd(g, (R)re);
                atomicAdd(g + 1, (R)im);
            }
            __syncthreads();  // the tile is reused by the next problem
        }
    }
}

// Charge density of mode m of the samples shifted along z, one plane per problem (sections 3.2, 3.5):
//   rho(z_i, rho_k) += q w S3(i - z'/dz) / dz * R_k * A_m,  z' = z + shift.
// DEP_PER_THREAD consecutive samples per thread; as for J_z, a block whose samples' shapes touch at most
// DEP_TILE cells of a problem sums its adds in an FP64 LDS tile and adds the tile to the plane once,
// otherwise every add is a global atomic.
template <typename R>
__global__ __launch_bounds__(256) void k_deposit_rho(DepositArgs A)
{
    __shared__ double tile[2 * DEP_TILE];
    __shared__ int red[16];
    const int64_t s0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * DEP_PER_THREAD;
    for (int p = 0; p < A.nprob; ++p) {
        const ProbDesc &D = A.probs[p];
        int fp[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};  // zmin, zmax, kmin, kmax
#pragma unroll
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            const int64_t s = s0 + u;
            if (s >= A.n) continue;
            const double zc = (A.samples[4 * s] + A.shift) / D.dz;
            if (!z_on_grid(D, zc)) continue;
            const double x = A.samples[4 * s + 1], y = A.samples[4 * s + 2];
            const int kc = (int)floor(sqrt(x * x + y * y) / D.dr);
            fp[0] = min(fp[0], (int)floor(zc) - 1);
            fp[1] = max(fp[1], (int)floor(zc) + 2);
            fp[2] = min(fp[2], max(kc - 3, 0));
            fp[3] = max(fp[3], min(kc + 3, D.nr - 1));
        }
        block_minmax(fp, red);
        if (fp[1] < fp[0]) continue;  // no sample of the block is deposited into this problem
        const int tz = fp[1] - fp[0] + 1, tr = fp[3] - fp[2] + 1;
        const bool use_tile = (int64_t)tz * tr <= DEP_TILE;  // uniform across the block
        R *rp = (R *)A.j[p];
        if (use_tile) {
            for (int c = threadIdx.x; c < 2 * tz * tr; c += 256) tile[c] = 0.0;
            __syncthreads();
        }
#pragma unroll 1
        for (int u = 0; u < DEP_PER_THREAD; ++u) {
            const int64_t s = s0 + u;
            if (s >= A.n) continue;
            const double z = A.samples[4 * s] + A.shift, x = A.samples[4 * s + 1], y = A.samples[4 * s + 2];
            const double qw = A.samples[4 * s + 3];
            const double zc = z / D.dz;
            if (!z_on_grid(D, zc)) continue;
            const double rho = sqrt(x * x + y * y);
            const int lo = (int)floor(zc) - 1;
            double wz[4];
            for (int v = 0; v < 4; ++v) wz[v] = bspline3(lo + v - zc) / D.dz;
            const SampleShape S = sample_shape(D, rho, x, y, A.eps, fold_mS(D.m));
#pragma unroll
            for (int jr = 0; jr < 7; ++jr) {
                const int k = S.kc - 3 + jr;
                const double rs = S.w[jr];
                if (rs == 0.0) continue;
                for (int v = 0; v < 4; ++v) {
                    const double w = qw * wz[v] * rs;
                    if (w == 0.0) continue;
                    if (use_tile) {
                        double *c = tile + 2 * ((k - fp[2]) * tz + lo + v - fp[0]);
                        atomicAdd(c, w * S.ar);
                        atomicAdd(c + 1, w * S.ai);
                    } else {
                        R *c = rp + 2 * ((size_t)k * D.nz + lo + v);
                        atomicAdd(c, (R)(w * S.ar));
                        atomicAdd(c + 1, (R)(w * S.ai));
                    }
                }
            }
        }
        if (use_tile) {
            __syncthreads();
            for (int c = threadIdx.x; c < tz * tr; c += 256) {
                const double re = tile[2 * c], im = tile[2 * c + 1];
                if (re == 0.0 && im == 0.0) continue;
                R *g = rp + 2 * ((size_t)(fp[2] + c / tz) * D.nz + fp[0] + c % tz);
                atomicAdd(g, (R)re);
                atomicAdd(g + 1, (R)im);
            }
            __syncthreads();  // the tile is reused by the next problem
        }
    }
}

// --------------------------------------------------------------------------------------------------
// Ponderomotive field of the envelope model (section 4.3), m = 0:
//   |a|^2,  A~_rho(k) = -sum_j a_j (I(k + j - 1) - I(k - j)) / dr (staggered rows k >= 1, row 0 = 0),
//   A~_z(i) = -sum_j a_j (I(i + j - 1) - I(i - j)) / dz (staggered columns);
// I = |a|^2 with rows below the axis mirrored (even), rows from nr on and columns outside the grid 0.
// Blocks of PON_Z columns x PON_R rows: I over the block and its N_D-wide halo is formed once into LDS,
// then each thread takes PON_R / 4 rows of one column.
// --------------------------------------------------------------------------------------------------
constexpr int PON_Z = 64, PON_R = 16;
template <typename R>
__global__ __launch_bounds__(256) void k_ponderomotive(const ProbDesc *Dp, const void *av, void *outv, int nd)
{
    using V = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
    constexpr int TW = PON_Z + 2 * kMaxND, TH = PON_R + 2 * kMaxND;
    __shared__ double T[TH * TW];
    const ProbDesc &D = *Dp;
    const int i0 = blockIdx.x * PON_Z, k0 = blockIdx.y * PON_R;
    const int tw = PON_Z + 2 * nd, th = PON_R + 2 * nd;  // tile: rows k0 - nd .., columns i0 - nd ..
    const V *a = (const V *)av;
    for (int e = threadIdx.x; e < tw * th; e += 256) {
        const int c = i0 - nd + e % tw, q = k0 - nd + e / tw;
        const int qq = q < 0 ? -1 - q : q;
        double v = 0.0;
        if (c >= 0 && c < D.nz && qq < D.nr) {
            const V x = a[(size_t)qq * D.nz + c];
            v = (double)x.x * (double)x.x + (double)x.y * (double)x.y;
        }
        T[(e / tw) * TW + e % tw] = v;
    }
    __syncthreads();
    const int ci = threadIdx.x % PON_Z, i = i0 + ci;
    if (i >= D.nz) return;
    R *out = (R *)outv;
    for (int r = threadIdx.x / PON_Z; r < PON_R; r += 256 / PON_Z) {
        const int k = k0 + r;
        if (k >= D.nr) break;
        auto I = [&](int dq, int dc) { return T[(r + nd + dq) * TW + ci + nd + dc]; };  // I(k + dq, i + dc)
        double gr = 0.0, gz = 0.0;
        for (int j = 1; j <= nd; ++j) {
            if (k >= 1) gr += D.ar[j - 1] * (I(j - 1, 0) - I(-j, 0));
            gz += D.az[j - 1] * (I(0, j - 1) - I(0, -j));
        }
        const size_t o = (size_t)k * D.nz + i;
        out[o] = (R)I(0, 0);
        out[D.plane + o] = (R)(-gr);
        out[2 * D.plane + o] = (R)(-gz);
    }
}

// --------------------------------------------------------------------------------------------------
// Current correction (section 3.7).  FP64 arithmetic throughout; J in the storage precision.
// --------------------------------------------------------------------------------------------------
template <typename R>
struct cplx_of { using V = double2; };
template <>
struct cplx_of<float> { using V = float2; };
template <typename V>
__device__ __forceinline__ double2 ld2(const V *p, size_t q)
{
    const V v = p[q];
    return double2{(double)v.x, (double)v.y};
}

// d(k, i) = rho_xy - rho_k^-1 sum_j a_j (g(k + j) - g(k - j + 1)) / dr - (i m / rho_k) J_theta,
// g(q) = q dr Jbar_rho(q) on the staggered rows, 0 on the axis, parity * g(-q) below it, 0 from nr on.
template <typename R>
__global__ __launch_bounds__(256) void k_corr_div(CorrectArgs A)
{
    using V = typename cplx_of<R>::V;
    const int i = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y;
    if (i >= A.nz) return;
    const V *jr = (const V *)A.jbar;
    auto g = [&](int q) -> double2 {
        if (q == 0 || q >= A.nr || -q >= A.nr) return double2{0.0, 0.0};
        const int qq = q < 0 ? -q : q;
        const double2 v = ld2(jr, (size_t)qq * A.nz + i);
        const double f = (q < 0 ? (double)A.parity : 1.0) * qq * A.dr;
        return double2{f * v.x, f * v.y};
    };
    double sx = 0.0, sy = 0.0;
    for (int j = 1; j <= A.nd; ++j) {
        const double2 p = g(k + j), q = g(k - j + 1);
        sx += A.a[j - 1] * (p.x - q.x);
        sy += A.a[j - 1] * (p.y - q.y);
    }
    const double rho = (k + 0.5) * A.dr;
    const size_t o = (size_t)k * A.nz + i;
    const double2 t = ld2((const V *)A.jth_in, o), r = ld2((const V *)A.rho_xy, o);
    const double mr = A.m / rho;
    // (i m / rho) (tx + i ty) = (-mr ty, mr tx)
    A.work[o] = double2{r.x - sx / (A.dr * rho) + mr * t.y, r.y - sy / (A.dr * rho) - mr * t.x};
}

// Lane `lane` of a double held across the wave, as a wave-uniform value (two v_readlane into scalars).
__device__ __forceinline__ double readlane_d(double x, int lane)
{
    const unsigned long long b = __builtin_bit_cast(unsigned long long, x);
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, lane);
    const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), lane);
    return __builtin_bit_cast(double, ((unsigned long long)hi << 32) | lo);
}

// Banded triangular solves of the current correction, one thread per z column and row segment.
// Forward: y_k = d_k - sum_j L(k, k-j) y_(k-j); backward: x_k = (y_k - sum_j U(k, k+j) x_(k+j)) / U(k, k).
// Boundary value t of a segment [a, b): forward y(a - 1 - t), backward x(b + t), t < N_D.
//
// k_seg_solve: each segment from a zero boundary, in place.  Every column uses the same factors: a
// wavefront loads those of a chunk of CH rows spread over its lanes and takes each as a wave-uniform
// scalar with v_readlane; two chunk buffers are refilled in place a chunk ahead (no register moves of
// loads in flight, so no wait covers the stores issued after them).  Loads read clamped rows
// unconditionally (a branch around a load would make the wave wait for it); words and values of rows
// outside the segment are never used.  Block (x, y, z): columns, problem y, segment z.
template <int ND>
__global__ __launch_bounds__(256) void k_seg_solve(SolveArgs S, int fwd)
{
    constexpr int CH = 16, W = 2 * ND + 1, WORDS = CH * W, NREG = (WORDS + 63) / 64;
    const auto &P = S.p[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x, lane = threadIdx.x % 64, sg = blockIdx.z;
    if (sg >= P.nseg || i - lane >= P.nz) return;  // the whole wavefront is idle
    const bool active = i < P.nz;                   // the others read column 0 and store nothing
    const int nr = P.nr, a = sg * P.seg, b = min(nr, a + P.seg), nchunk = (b - a + CH - 1) / CH;
    const size_t nz = (size_t)P.nz;
    double2 *col = P.work + (active ? i : 0);
    const double *band = P.band;
    auto row_of = [&](int c, int r) { return fwd ? a + c * CH + r : b - 1 - c * CH - r; };
    auto clamp_row = [&](int k) { return k < 0 ? 0 : (k >= nr ? nr - 1 : k); };
    auto load = [&](int c, double2 (&v)[CH], double (&w)[NREG]) {
#pragma unroll
        for (int u = 0; u < NREG; ++u) {
            const int e = lane + 64 * u;
            const int ec = e < WORDS ? e : WORDS - 1;
            w[u] = band[(size_t)clamp_row(row_of(c, ec / W)) * W + ec % W];
        }
#pragma unroll
        for (int r = 0; r < CH; ++r) v[r] = col[clamp_row(row_of(c, r)) * nz];
    };
    double2 win[ND];
#pragma unroll
    for (int t = 0; t < ND; ++t) win[t] = double2{0.0, 0.0};  // forward: y(k - 1 - t); backward: x(k + 1 + t)
    auto solve = [&](int c, const double2 (&vals)[CH], const double (&cw)[NREG]) {
#pragma unroll
        for (int r = 0; r < CH; ++r) {
            const int k = row_of(c, r);
            if (k < a || k >= b) continue;  // uniform: the same rows for every lane
            auto coef = [&](int t) { return readlane_d(cw[(r * W + t) / 64], (r * W + t) % 64); };
            // the older taps first, in two partial sums; the newest value enters last
            double2 v = vals[r], h = double2{0.0, 0.0};
#pragma unroll
            for (int j = ND; j >= 2; --j) {
                const double f = coef(fwd ? ND - j : ND + j);  // L(k, k - j) or U(k, k + j)
                double2 &acc = (j & 1) ? v : h;
                acc.x -= f * win[j - 1].x;
                acc.y -= f * win[j - 1].y;
            }
            v.x += h.x;
            v.y += h.y;
            const double f1 = coef(fwd ? ND - 1 : ND + 1);
            v.x -= f1 * win[0].x;
            v.y -= f1 * win[0].y;
            if (!fwd) {
                const double d = coef(ND);
                v.x *= d;
                v.y *= d;
            }
            if (active) col[k * nz] = v;
#pragma unroll
            for (int t = ND - 1; t > 0; --t) win[t] = win[t - 1];
            win[0] = v;
        }
    };
    double2 va[CH], vb[CH];
    double wa[NREG], wb[NREG];
    load(0, va, wa);
    for (int c = 0; c < nchunk; c += 2) {
        load(c + 1, vb, wb);
        solve(c, va, wa);
        load(c + 2, va, wa);
        if (c + 1 < nchunk) solve(c + 1, vb, wb);
    }
}

// k_seg_fix: a group of GS >= N_D lanes per column (lane t forms boundary value t) sweeps the segments in
// the order of the pass and writes the true boundary values of each (but the first) to wbuf: those of the
// segment before it (forward) or after it (backward), formed as the zero-start value plus that segment's
// response to its own boundary values, which the group exchanges by lane shuffles.  The zero-start value
// of the next segment is loaded a step ahead.
constexpr int seg_fix_group(int nd) { return nd <= 1 ? 1 : nd <= 2 ? 2 : nd <= 4 ? 4 : nd <= 8 ? 8 : 16; }
template <int ND>
__global__ __launch_bounds__(256) void k_seg_fix(SolveArgs S, int fwd)
{
    constexpr int GS = seg_fix_group(ND);
    const auto &P = S.p[blockIdx.y];
    const int t = threadIdx.x % GS, base = (threadIdx.x % 64) - t;  // lane of boundary value 0 of the group
    const int i = blockIdx.x * (256 / GS) + threadIdx.x / GS;
    if (i >= P.nz) return;  // the whole group: shuffles only read lanes of the same column
    const int nr = P.nr, seg = P.seg, ns = P.nseg;
    const size_t nz = (size_t)P.nz;
    const double *G = fwd ? P.gf : P.gb;
    auto row_of = [&](int step) {  // row of boundary value t of the segment formed at this step
        const int sg = fwd ? step : ns - 1 - step;
        return fwd ? sg * seg - 1 - t : (sg + 1) * seg + t;
    };
    auto load = [&](int step) {
        const int k = row_of(step);
        return (t < ND && step < ns && k >= 0 && k < nr) ? P.work[(size_t)k * nz + i] : double2{0.0, 0.0};
    };
    double2 w = double2{0.0, 0.0};  // this lane's boundary value of the segment the sweep has just passed
    double2 next = load(1);
    for (int step = 1; step < ns; ++step) {
        const int sg = fwd ? step : ns - 1 - step;   // segment whose boundary values are formed
        const int src = fwd ? sg - 1 : sg + 1;        // the segment they lie in
        const bool src_has = fwd ? src >= 1 : src <= ns - 2;  // src itself has boundary values
        const int k = row_of(step);
        double2 v = next;
        next = load(step + 1);
        if (src_has) {  // + response row of this value to the group's previous values
#pragma unroll
            for (int u = 0; u < ND; ++u) {
                const double wx = __shfl(w.x, base + u, 64), wy = __shfl(w.y, base + u, 64);
                const double g = (t < ND && k >= 0 && k < nr) ? G[(size_t)k * ND + u] : 0.0;
                v.x += g * wx;
                v.y += g * wy;
            }
        }
        w = v;
        if (t < ND) P.wbuf[((size_t)sg * ND + t) * nz + i] = v;
    }
}

// k_seg_apply: rows of every segment but the first of the pass += response x boundary values.  One thread
// per column and chunk of SEG_APPLY_ROWS rows of a segment (blockIdx.z = segment * chunks + chunk); the
// chunk's loads are issued before its stores.
constexpr int SEG_APPLY_ROWS = 8;
template <int ND>
__global__ __launch_bounds__(256) void k_seg_apply(SolveArgs S, int fwd, int chunks)
{
    const auto &P = S.p[blockIdx.y];
    const int i = blockIdx.x * 256 + threadIdx.x, sg = blockIdx.z / chunks, ch = blockIdx.z % chunks;
    if (sg >= P.nseg || i >= P.nz || sg == (fwd ? 0 : P.nseg - 1)) return;
    const int a = sg * P.seg + ch * SEG_APPLY_ROWS, b = min(min(P.nr, (sg + 1) * P.seg), a + SEG_APPLY_ROWS);
    if (a >= b) return;
    const size_t nz = (size_t)P.nz;
    const double *G = fwd ? P.gf : P.gb;
    double2 w[ND];
#pragma unroll
    for (int t = 0; t < ND; ++t) w[t] = P.wbuf[((size_t)sg * ND + t) * nz + i];
    double2 v[SEG_APPLY_ROWS];
#pragma unroll
    for (int c = 0; c < SEG_APPLY_ROWS; ++c) v[c] = a + c < b ? P.work[(size_t)(a + c) * nz + i] : double2{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < SEG_APPLY_ROWS; ++c) {
        const int k = min(a + c, b - 1);
#pragma unroll
        for (int u = 0; u < ND; ++u) {
            const double g = G[(size_t)k * ND + u];
            v[c].x += g * w[u].x;
            v[c].y += g * w[u].y;
        }
    }
#pragma unroll
    for (int c = 0; c < SEG_APPLY_ROWS; ++c)
        if (a + c < b) P.work[(size_t)(a + c) * nz + i] = v[c];
}

// Jbar_rho(k) += sum_j a_j (phi(k + j - 1) - phi(k - j)) / dr on the staggered rows k >= 1 (phi on the
// primary rows, parity * phi(-1-q) below the axis, 0 from nr on);  J_theta~ = J_theta + (i m / rho) phi.
template <typename R>
__global__ __launch_bounds__(256) void k_corr_apply(CorrectArgs A)
{
    using V = typename cplx_of<R>::V;
    const int i = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y;
    if (i >= A.nz) return;
    auto phi = [&](int q) -> double2 {
        const int qq = q < 0 ? -1 - q : q;
        if (qq >= A.nr) return double2{0.0, 0.0};
        const double2 v = A.work[(size_t)qq * A.nz + i];
        const double sg = q < 0 ? (double)A.parity : 1.0;
        return double2{sg * v.x, sg * v.y};
    };
    const size_t o = (size_t)k * A.nz + i;
    if (k >= 1) {
        double sx = 0.0, sy = 0.0;
        for (int j = 1; j <= A.nd; ++j) {
            const double2 p = phi(k + j - 1), q = phi(k - j);
            sx += A.a[j - 1] * (p.x - q.x);
            sy += A.a[j - 1] * (p.y - q.y);
        }
        V *jr = (V *)A.jbar;
        const double2 v = ld2(jr, o);
        jr[o] = V{(R)(v.x + sx / A.dr), (R)(v.y + sy / A.dr)};
    }
    const double mr = A.m / ((k + 0.5) * A.dr);
    const double2 t = ld2((const V *)A.jth_in, o), f = A.work[o];
    ((V *)A.jth_out)[o] = V{(R)(t.x - mr * f.y), (R)(t.y + mr * f.x)};
}

// --------------------------------------------------------------------------------------------------
// Field interpolation (section 3.3).  Destaggering, one thread per output cell of the samples' footprint
// box (rows grown by the reach of a later pass), grid-stride, up to six independent passes per launch;
// the other cells are not written:
//   along z:   out(k, i) = sum_j s_j (f(k, i + j) + f(k, i - j + 1)),  columns outside [0, nz) are 0;
//   along rho: out(k, i) = sum_j s_j (f(k + j, i) + f(k - j + 1, i)) on the staggered rows, row 0 = the
//              axis value (sum_k' c_k' f(k', i) when extrapolated, else 0), rows q < 0 = parity f(-q),
//              rows >= nr are 0.  FP64 arithmetic, storage precision in and out.
// 2x supersampling also shifts the other way (to_stag), primary to staggered positions:
//   along z:   out(k, i) = sum_j s_j (f(k, i + j - 1) + f(k, i - j)),
//   along rho: out(k, i) = sum_j s_j (f(k + j - 1, i) + f(k - j, i)) for every k >= 0, rows q < 0 =
//              parity f(-1-q),
// copies the stored sets (the axis row of a staggered-rho set by the axis rule), and writes the axis row
// of a z-shifted staggered-rho set by the axis rule in place.
// --------------------------------------------------------------------------------------------------
// The footprint box of the samples: a grid-stride pass whose blocks store their partial boxes, then one
// block that reduces them (no same-address atomics).
__global__ __launch_bounds__(256) void k_gather_box(const double *samples, int64_t n, int nz, int nr, double dz,
                                                    double dr, int *part)
{
    __shared__ int red[16];
    int v[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    for (int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x; s < n; s += (int64_t)gridDim.x * 256) {
        const double z = samples[4 * s], x = samples[4 * s + 1], y = samples[4 * s + 2];
        const double zc = z / dz, rc = sqrt(x * x + y * y) / dr - 0.5;
        // shapes over nodes floor(zc) - 1 .. + 2 and rows floor(rc) - 1 .. + 2 (rows below the axis read
        // rows 0 and 1); far-away samples are clamped, their shape reads nothing
        const double zf = fmin(fmax(floor(zc), -4.0), (double)nz + 4.0), rf = fmin(floor(rc), (double)nr + 4.0);
        const int a = max(0, (int)zf - 1), b = min(nz - 1, (int)zf + 2);
        if (a > b) continue;
        v[0] = min(v[0], a);
        v[1] = max(v[1], b);
        v[2] = min(v[2], max(0, (int)rf - 1));
        v[3] = max(v[3], min(nr - 1, max(1, (int)rf + 2)));
    }
    block_minmax(v, red);
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = v[threadIdx.x];
}
__global__ __launch_bounds__(256) void k_gather_box_reduce(const int *part, int nblocks, int *box)
{
    __shared__ int red[16];
    int v[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    for (int b = threadIdx.x; b < nblocks; b += 256) {
        v[0] = min(v[0], part[4 * b]);
        v[1] = max(v[1], part[4 * b + 1]);
        v[2] = min(v[2], part[4 * b + 2]);
        v[3] = max(v[3], part[4 * b + 3]);
    }
    block_minmax(v, red);
    if (threadIdx.x < 4) box[threadIdx.x] = v[threadIdx.x];
}

template <typename R>
__global__ __launch_bounds__(256) void k_destagger(DestaggerArgs A)
{
    using V = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
    const DestaggerPass &P = A.pass[blockIdx.y];
    const int nd = A.nd[P.set];
    const double *sw = A.s[P.set], *cw = A.c[P.set];
    // the cells of the box (rows grown by grow_r), grid-stride
    const int z0 = max(0, A.box[0]), z1 = min(A.nz - 1, A.box[1]);
    const int k0 = max(0, A.box[2] - P.grow_r);
    int k1 = min(A.nr - 1, A.box[3] + P.grow_r);
    if (P.op == PASS_AXIS) {
        if (k0 > 0) return;  // the box does not reach the axis
        k1 = 0;
    }
    if (z1 < z0 || k1 < k0) return;
    const int64_t w = z1 - z0 + 1, cells = w * (int64_t)(k1 - k0 + 1);
    const V *f = (const V *)P.src;
    auto at = [&](int q, int col) -> double2 {
        const V v = f[(size_t)q * A.nz + col];
        return double2{(double)v.x, (double)v.y};
    };
    for (int64_t cell = (int64_t)blockIdx.x * 256 + threadIdx.x; cell < cells; cell += (int64_t)gridDim.x * 256) {
        const int i = z0 + (int)(cell % w), k = k0 + (int)(cell / w);
        // Taps outside the grid read a clamped in-range value with weight 0 (loads need no branches and can
        // all be in flight together); the sums are the same.
        double re = 0.0, im = 0.0;
        if (P.op == PASS_COPY || P.op == PASS_AXIS) {
            if (k == 0 && (P.axis_rule || P.op == PASS_AXIS)) {
                if (P.extrapolate)
                    for (int q = 1; q <= nd && q < A.nr; ++q) {
                        const double2 v = at(q, i);
                        re += cw[q - 1] * v.x;
                        im += cw[q - 1] * v.y;
                    }
            } else {
                const double2 v = at(k, i);
                re = v.x;
                im = v.y;
            }
        } else if (P.op == PASS_Z) {
#pragma unroll 4
            for (int j = 1; j <= nd; ++j) {
                const int c0 = i + j - P.to_stag, c1 = i - j + 1 - P.to_stag;
                const double2 v0 = at(k, min(c0, A.nz - 1)), v1 = at(k, max(c1, 0));
                const double w0 = c0 < A.nz ? sw[j - 1] : 0.0, w1 = c1 >= 0 ? sw[j - 1] : 0.0;
                re += w0 * v0.x;
                im += w0 * v0.y;
                re += w1 * v1.x;
                im += w1 * v1.y;
            }
        } else if (P.to_stag) {
            // primary rows k + j - 1 and k - j to the staggered row k (the axis for k = 0); rows below the
            // axis mirror row -1-q with the parity, rows >= nr are 0
#pragma unroll 4
            for (int j = 1; j <= nd; ++j) {
                const int q0 = k + j - 1, q1 = k - j, a1 = q1 < 0 ? -1 - q1 : q1;
                const double2 v0 = at(min(q0, A.nr - 1), i), v1 = at(min(a1, A.nr - 1), i);
                const double g0 = q0 < A.nr ? 1.0 : 0.0, g1 = a1 >= A.nr ? 0.0 : (q1 < 0 ? (double)P.parity : 1.0);
                re += sw[j - 1] * (g0 * v0.x + g1 * v1.x);
                im += sw[j - 1] * (g0 * v0.y + g1 * v1.y);
            }
        } else {
            double axr = 0.0, axi = 0.0;
            if (P.extrapolate)
                for (int q = 1; q <= nd && q < A.nr; ++q) {
                    const double2 v = at(q, i);
                    axr += cw[q - 1] * v.x;
                    axi += cw[q - 1] * v.y;
                }
            // row q of the extended grid: 0 beyond the last row, the axis value on row 0, parity * row -q
            // below the axis
#pragma unroll 4
            for (int j = 1; j <= nd; ++j) {
                const int q0 = k + j, q1 = k - j + 1, a1 = q1 < 0 ? -q1 : q1;
                const double2 v0 = at(min(q0, A.nr - 1), i), v1 = at(min(a1, A.nr - 1), i);
                const double g0 = q0 < A.nr ? 1.0 : 0.0, g1 = a1 >= A.nr ? 0.0 : (q1 < 0 ? (double)P.parity : 1.0);
                const double x0 = g0 * v0.x, y0 = g0 * v0.y;
                const double x1 = q1 == 0 ? axr : g1 * v1.x, y1 = q1 == 0 ? axi : g1 * v1.y;
                re += sw[j - 1] * (x0 + x1);
                im += sw[j - 1] * (y0 + y1);
            }
        }
        ((V *)P.dst)[(size_t)k * A.nz + i] = V{(R)re, (R)im};
    }
}

// Interpolation, one thread per sample: for each mode m and component c,
//   Re( e^(i m theta) sum_(i,k) S3(i - z/dz) S3(k + 1/2 - rho/drho) F_c(k, i) )
// over the extended primary grid (rows k < 0 take parity * row -1-k: m_A for the rho and theta
// components, m_S for the z ones; rows >= nr and columns outside the grid are 0), summed over the modes.
// Blocks take GATHER_BLOCK consecutive samples; two blocks share a CU, so one block's loads overlap the
// other's arithmetic.  When the nodes and rows their shapes touch (rows below the axis read rows 0 and 1)
// fit GATHER_TILE values over all modes and components, the block first copies them into LDS (as FP64)
// and every sample reads its 16 nodes per mode and component from there; position-ordered samples make
// that footprint small.  Otherwise the samples read the planes directly.
constexpr int GATHER_BLOCK = 512, GATHER_TILE = 4096;
template <typename R>
__global__ __launch_bounds__(GATHER_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_gather(GatherArgs A)
{
    using V = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
    __shared__ double2 tile[GATHER_TILE];
    __shared__ int red[4 * (GATHER_BLOCK / 64)];
    const int64_t s = (int64_t)blockIdx.x * GATHER_BLOCK + threadIdx.x;
    const bool live = s < A.n;
    double z = 0.0, x = 0.0, y = 0.0;
    if (live) {
        z = A.samples[4 * s];
        x = A.samples[4 * s + 1];
        y = A.samples[4 * s + 2];
    }
    const double rho = sqrt(x * x + y * y);
    // footprint of the block's samples: the nodes inside the grid that their stencils touch
    int fp[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    {
        const double zf = fmin(fmax(floor(z / A.dz), -4.0), (double)A.nz + 4.0);
        const double rf = fmin(floor(rho / A.dr - 0.5), (double)A.nr + 4.0);
        const int a = max(0, (int)zf - 1), b = min(A.nz - 1, (int)zf + 2);
        if (live && a <= b) {
            fp[0] = a;
            fp[1] = b;
            fp[2] = max(0, (int)rf - 1);
            fp[3] = min(A.nr - 1, max(1, (int)rf + 2));
        }
    }
    block_minmax<GATHER_BLOCK / 64>(fp, red);
    // Tile rows are ts = tz | 1 values apart: an odd stride puts 16 consecutive rows in distinct LDS bank
    // groups of 16-byte reads, and the lanes of a wave (samples at about the same z) differ mostly in row.
    const bool any = fp[1] >= fp[0] && fp[3] >= fp[2];  // some sample of the block touches the grid
    const int tz = any ? fp[1] - fp[0] + 1 : 0, tr = any ? fp[3] - fp[2] + 1 : 0, ts = tz | 1;
    const bool use_tile = any && (int64_t)ts * tr * 6 * A.nprob <= GATHER_TILE;  // uniform
    if (use_tile) {
        const int per = tz * tr, total = per * 6 * A.nprob;
        for (int e = threadIdx.x; e < total; e += GATHER_BLOCK) {
            const int pc = e / per, cell = e % per, k = cell / tz, i = cell % tz;
            const V v = ((const V *)A.plane[pc / 6][pc % 6])[(size_t)(fp[2] + k) * A.nz + fp[0] + i];
            tile[(pc * tr + k) * ts + i] = double2{(double)v.x, (double)v.y};
        }
        __syncthreads();
    }
    if (!live) return;
    // e^(i theta) from the position itself (theta = 0 on the axis); e^(i m theta) is its m-th power
    const double c1 = rho > 0.0 ? x / rho : 1.0, s1 = rho > 0.0 ? y / rho : 0.0;
    const double zc = z / A.dz, rc = rho / A.dr - 0.5;
    const int i0 = (int)floor(zc) - 1, k0 = (int)floor(rc) - 1;
    // Nodes outside the grid get weight zero and an index clamped into the tile (or the plane), so every
    // read stays in bounds and the loops need no branches; the mirrored rows below the axis take the
    // component's parity as a sign.
    const int zlo = use_tile ? fp[0] : 0, zhi = use_tile ? fp[1] : A.nz - 1;
    const int rlo = use_tile ? fp[2] : 0, rhi = use_tile ? fp[3] : A.nr - 1;
    double wz[4], wr[4];
    int col[4], row[4];
    bool below[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + v, k = k0 + v, q = k < 0 ? -1 - k : k;
        wz[v] = (i >= 0 && i < A.nz) ? bspline3(i - zc) : 0.0;
        wr[v] = q < A.nr ? bspline3(k - rc) : 0.0;
        col[v] = min(max(i, zlo), zhi) - zlo;
        row[v] = min(max(q, rlo), rhi) - rlo;
        below[v] = k < 0;
    }
#pragma unroll 1
    for (int c = 0; c < 6; ++c) {
        double acc = 0.0;
        for (int p = 0; p < A.nprob; ++p) {
            const int m = A.m[p];
            const double pS = (m % 2 == 0) ? 1.0 : -1.0, pA = ((m > 1 ? m - 1 : 1 - m) % 2 == 0) ? 1.0 : -1.0;
            const double par = (c == 2 || c == 5) ? pS : pA;
            double cr = 1.0, ci = 0.0;
            for (int j = 0; j < (m < 0 ? -m : m); ++j) {
                const double t = cr * c1 - ci * s1;
                ci = cr * s1 + ci * c1;
                cr = t;
            }
            if (m < 0) ci = -ci;
            double re = 0.0, im = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                const double wa = below[a] ? par * wr[a] : wr[a];
                double v[8];
                if (use_tile) {
                    const double2 *t = tile + ((p * 6 + c) * tr + row[a]) * ts;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double2 g = t[col[b]];
                        v[2 * b] = g.x;
                        v[2 * b + 1] = g.y;
                    }
                } else {
                    const V *f = (const V *)A.plane[p][c] + (size_t)row[a] * A.nz;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const V g = f[col[b]];
                        v[2 * b] = g.x;
                        v[2 * b + 1] = g.y;
                    }
                }
                double rre = 0.0, rim = 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    rre += wz[b] * v[2 * b];
                    rim += wz[b] * v[2 * b + 1];
                }
                re += wa * rre;
                im += wa * rim;
            }
            acc += re * cr - im * ci;
        }
        A.fields[6 * s + c] = acc;
    }
}

// Interpolation on the doubled grid (2x supersampling, section 3.4; SS bit 0: z, bit 1: rho), one thread
// per sample.  Doubled along z the nodes are u dz/2 (odd u: staggered column (u+1)/2, even u: primary
// column u/2); doubled along rho they are g drho/2 (even g: staggered row g/2, the axis for g = 0; odd g:
// primary row (g-1)/2; g < 0 the mirror of -g with the parity); a direction not doubled keeps the primary
// nodes.  The cubic shape is in units of the node spacing.  Every position set is read from the doubled-
// grid planes (their axis rows already hold the axis rule where it applies).  Blocks of GATHER_BLOCK
// consecutive samples go mode by mode: when the columns and rows the block's nodes touch fit GATHER_TILE
// values over the mode's position sets and components, the block copies them into LDS first; otherwise
// the samples read the planes.  Each mode's value is added into fields in mode order.
template <typename R, int SS>
__global__ __launch_bounds__(GATHER_BLOCK) __attribute__((amdgpu_waves_per_eu(4))) void k_gather_fine(GatherArgs A)
{
    using V = typename std::conditional<std::is_same<R, double>::value, double2, float2>::type;
    constexpr int NSET = SS == 3 ? 4 : 2;  // position sets the doubled grid reads per component
    __shared__ double2 tile[GATHER_TILE];
    __shared__ int red[4 * (GATHER_BLOCK / 64)];
    const int64_t s = (int64_t)blockIdx.x * GATHER_BLOCK + threadIdx.x;
    const bool live = s < A.n;
    double z = 0.0, x = 0.0, y = 0.0;
    if (live) {
        z = A.samples[4 * s];
        x = A.samples[4 * s + 1];
        y = A.samples[4 * s + 2];
    }
    const double rho = sqrt(x * x + y * y);
    const double c1 = rho > 0.0 ? x / rho : 1.0, s1 = rho > 0.0 ? y / rho : 0.0;
    double wz[4], wr[4];
    int col[4], row[4], zsb[4], rsb[4];
    bool below[4];
    int fp[4] = {INT_MAX, INT_MIN, INT_MAX, INT_MIN};
    {
        const double zc = (SS & 1) ? 2.0 * z / A.dz : z / A.dz;
        const int u0 = (int)floor(zc) - 1;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int u = u0 + b, zs = (SS & 1) ? (u & 1) : 0, i = (SS & 1) ? (u + zs) >> 1 : u;
            const bool ok = i >= 0 && i < A.nz;
            wz[b] = ok ? bspline3(u - zc) : 0.0;
            col[b] = min(max(i, 0), A.nz - 1);
            zsb[b] = zs;
            if (live && ok) {
                fp[0] = min(fp[0], i);
                fp[1] = max(fp[1], i);
            }
        }
        const double rc = (SS & 2) ? 2.0 * rho / A.dr : rho / A.dr - 0.5;
        const int g0 = (int)floor(rc) - 1;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const int g = g0 + a;
            int rs, k;
            if (SS & 2) {
                const int gg = g < 0 ? -g : g;
                rs = (gg & 1) ? 0 : 1;
                k = rs ? gg >> 1 : (gg - 1) >> 1;
            } else {
                rs = 0;
                k = g < 0 ? -1 - g : g;
            }
            const bool ok = k < A.nr;
            wr[a] = ok ? bspline3(g - rc) : 0.0;
            row[a] = min(k, A.nr - 1);
            rsb[a] = rs;
            below[a] = g < 0;
            if (live && ok) {
                fp[2] = min(fp[2], k);
                fp[3] = max(fp[3], k);
            }
        }
    }
    block_minmax<GATHER_BLOCK / 64>(fp, red);
    const bool any = fp[1] >= fp[0] && fp[3] >= fp[2];  // some sample of the block touches the grid
    const int tz = any ? fp[1] - fp[0] + 1 : 0, tr = any ? fp[3] - fp[2] + 1 : 0, ts = tz | 1;
    const bool use_tile = any && (int64_t)NSET * 6 * tr * ts <= GATHER_TILE;  // uniform
    // Offset of each node within a component's values: in the tile (slot of the position set, then row and
    // column, nodes outside the grid -- weight 0 -- clamped into the tile), or in its four doubled-grid
    // planes (set, row, column; the planes of one component span less than 2^31 values).
    int off[4][4];
    const int cells = A.nz * A.nr;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int v = zsb[b] + 2 * rsb[a];
            if (use_tile) {
                const int t = SS == 1 ? (v & 1) : (SS == 2 ? (v >> 1) : v);
                off[a][b] = (t * tr + min(max(row[a], fp[2]), fp[3]) - fp[2]) * ts + min(max(col[b], fp[0]), fp[1]) - fp[0];
            } else {
                off[a][b] = v * cells + row[a] * A.nz + col[b];
            }
        }
    for (int p = 0; p < A.nprob; ++p) {
        const char *fine = (const char *)A.fine[p];
        if (use_tile) {
            if (p > 0) __syncthreads();  // the previous mode's reads are done
            const int per = tr * tz, total = NSET * 6 * per;
            for (int e = threadIdx.x; e < total; e += GATHER_BLOCK) {
                const int cs = e / per, cell = e % per, k = cell / tz, i = cell % tz;
                const int c = cs / NSET, t = cs % NSET;
                const int v = SS == 1 ? t : (SS == 2 ? 2 * t : t);
                const V g = ((const V *)(fine + (size_t)(4 * c + v) * A.plane_bytes))[(size_t)(fp[2] + k) * A.nz + fp[0] + i];
                tile[(cs * tr + k) * ts + i] = double2{(double)g.x, (double)g.y};
            }
            __syncthreads();
        }
        if (!live) continue;
        const int m = A.m[p];
        const double pS = (m % 2 == 0) ? 1.0 : -1.0, pA = ((m > 1 ? m - 1 : 1 - m) % 2 == 0) ? 1.0 : -1.0;
        double cr = 1.0, ci = 0.0;
        for (int j = 0; j < (m < 0 ? -m : m); ++j) {
            const double t = cr * c1 - ci * s1;
            ci = cr * s1 + ci * c1;
            cr = t;
        }
        if (m < 0) ci = -ci;
#pragma unroll 1
        for (int c = 0; c < 6; ++c) {
            const double par = (c == 2 || c == 5) ? pS : pA;
            const double2 *tc = tile + c * NSET * tr * ts;
            const V *gc = (const V *)(fine + (size_t)(4 * c) * A.plane_bytes);
            double re = 0.0, im = 0.0;
            auto sum = [&](auto fetch) {
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const double wa = below[a] ? par * wr[a] : wr[a];
                    double rre = 0.0, rim = 0.0;
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        const double2 g = fetch(off[a][b]);
                        rre += wz[b] * g.x;
                        rim += wz[b] * g.y;
                    }
                    re += wa * rre;
                    im += wa * rim;
                }
            };
            if (use_tile) sum([&](int o) { return tc[o]; });
            else sum([&](int o) {
                const V g = gc[o];
                return double2{(double)g.x, (double)g.y};
            });
            const double val = re * cr - im * ci;
            A.fields[6 * s + c] = p == 0 ? val : A.fields[6 * s + c] + val;
        }
    }
}

// Ponderomotive fields at samples (section 4.3).  First A~_rho and A~_z are brought to the primary grid,
// one thread per cell (S_rho^(+) from the staggered rows, odd, 0 on the axis; S_z^(+) from the staggered
// columns, 0 outside the grid; FP64), then one thread per sample interpolates |a|^2 and the two primary
// planes with the cubic shapes over the grid extended below the axis (|a|^2 and A~_z even, A~_rho odd),
// as k_gather does for m = 0.
template <typename R>
__global__ __launch_bounds__(256) void k_envelope_destagger(EnvGatherArgs A)
{
    const int i = blockIdx.x * 256 + threadIdx.x, k = blockIdx.y;
    if (i >= A.nz) return;
    const size_t plane = (size_t)A.nz * A.nr;
    const R *Ar = (const R *)A.pond + plane, *Az = (const R *)A.pond + 2 * plane;
    auto arow = [&](int r) -> double {  // A~_rho on staggered row r: 0 on the axis and from nr on
        const int a = r < 0 ? -r : r;
        if (r == 0 || a >= A.nr) return 0.0;
        const double v = (double)Ar[(size_t)a * A.nz + i];
        return r < 0 ? -v : v;
    };
    auto zcol = [&](int c) -> double { return (c < 0 || c >= A.nz) ? 0.0 : (double)Az[(size_t)k * A.nz + c]; };
    double vr = 0.0, vz = 0.0;
    for (int j = 1; j <= A.nd; ++j) {
        vr += A.s[j - 1] * (arow(k + j) + arow(k - j + 1));
        vz += A.s[j - 1] * (zcol(i + j) + zcol(i - j + 1));
    }
    A.prim[(size_t)k * A.nz + i] = vr;
    A.prim[plane + (size_t)k * A.nz + i] = vz;
}

template <typename R>
__global__ __launch_bounds__(256) void k_envelope_gather(EnvGatherArgs A)
{
    const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (q >= A.n) return;
    const double z = A.samples[4 * q], x = A.samples[4 * q + 1], y = A.samples[4 * q + 2];
    const double rho = sqrt(x * x + y * y);
    const size_t plane = (size_t)A.nz * A.nr;
    const R *I = (const R *)A.pond;
    const double *Pr = A.prim, *Pz = A.prim + plane;
    const double zc = z / A.dz, rc = rho / A.dr - 0.5;
    const int i0 = (int)floor(zc) - 1, k0 = (int)floor(rc) - 1;
    double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
    for (int a = 0; a < 4; ++a) {
        const int k = k0 + a, kk = k < 0 ? -1 - k : k;
        if (kk >= A.nr) continue;
        const double wr = bspline3(k - rc), sg = k < 0 ? -1.0 : 1.0;  // row k at (k + 1/2) drho
        if (wr == 0.0) continue;
        for (int b = 0; b < 4; ++b) {
            const int i = i0 + b;
            if (i < 0 || i >= A.nz) continue;
            const double wz = bspline3(i - zc);
            if (wz == 0.0) continue;
            const size_t o = (size_t)kk * A.nz + i;
            acc0 += wz * wr * (double)I[o];
            acc1 += wz * wr * (sg * Pr[o]);
            acc2 += wz * wr * Pz[o];
        }
    }
    A.out[3 * q] = acc0;
    A.out[3 * q + 1] = acc1;
    A.out[3 * q + 2] = acc2;
}

}  // namespace

hipError_t launch_envelope_gather(int prec, const EnvGatherArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (a.nd < 1 || a.nd > kMaxND || !a.prim) return hipErrorInvalidValue;
    const dim3 cells((unsigned)((a.nz + 255) / 256), (unsigned)a.nr), grid((unsigned)((a.n + 255) / 256));
    if (prec == P64) {
        hipLaunchKernelGGL(k_envelope_destagger<double>, cells, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_envelope_gather<double>, grid, dim3(256), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_envelope_destagger<float>, cells, dim3(256), 0, s, a);
        hipLaunchKernelGGL(k_envelope_gather<float>, grid, dim3(256), 0, s, a);
    }
    return hipGetLastError();
}

hipError_t launch_ponderomotive(int prec, const ProbDesc *d, int nz, int nr, int nd, const void *a, void *out,
                                hipStream_t s)
{
    if (nd < 1 || nd > kMaxND) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((nz + PON_Z - 1) / PON_Z), (unsigned)((nr + PON_R - 1) / PON_R));
    if (prec == P64) hipLaunchKernelGGL(k_ponderomotive<double>, grid, dim3(256), 0, s, d, a, out, nd);
    else hipLaunchKernelGGL(k_ponderomotive<float>, grid, dim3(256), 0, s, d, a, out, nd);
    return hipGetLastError();
}

hipError_t launch_correct_div(int prec, const CorrectArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.nz + 255) / 256), (unsigned)a.nr);
    if (prec == P64) hipLaunchKernelGGL(k_corr_div<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_corr_div<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_correct_apply(int prec, const CorrectArgs &a, hipStream_t s)
{
    const dim3 grid((unsigned)((a.nz + 255) / 256), (unsigned)a.nr);
    if (prec == P64) hipLaunchKernelGGL(k_corr_apply<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_corr_apply<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

template <int ND>
hipError_t correct_solve_nd(const SolveArgs &a, hipStream_t s)
{
    int nzmax = 0;
    for (int p = 0; p < a.nprob; ++p) nzmax = a.p[p].nz > nzmax ? a.p[p].nz : nzmax;
    const unsigned bx = (unsigned)((nzmax + 255) / 256);
    int segmax = 0;
    for (int p = 0; p < a.nprob; ++p) segmax = a.p[p].seg > segmax ? a.p[p].seg : segmax;
    const int chunks = (segmax + SEG_APPLY_ROWS - 1) / SEG_APPLY_ROWS;
    const dim3 seg(bx, (unsigned)a.nprob, (unsigned)a.smax), app(bx, (unsigned)a.nprob, (unsigned)(a.smax * chunks));
    constexpr int per = 256 / seg_fix_group(ND);  // columns per block of k_seg_fix
    const dim3 fix((unsigned)((nzmax + per - 1) / per), (unsigned)a.nprob);
    for (int fwd = 1; fwd >= 0; --fwd) {
        hipLaunchKernelGGL(k_seg_solve<ND>, seg, dim3(256), 0, s, a, fwd);
        if (a.smax > 1) {
            hipLaunchKernelGGL(k_seg_fix<ND>, fix, dim3(256), 0, s, a, fwd);
            hipLaunchKernelGGL(k_seg_apply<ND>, app, dim3(256), 0, s, a, fwd, chunks);
        }
    }
    return hipGetLastError();
}

hipError_t launch_correct_solve(const SolveArgs &a, hipStream_t s)
{
    if (a.nprob <= 0) return hipSuccess;
    switch (a.nd) {
#define C_(N) \
    case N: return correct_solve_nd<N>(a, s);
        C_(1) C_(2) C_(3) C_(4) C_(5) C_(6) C_(7) C_(8) C_(9) C_(10) C_(11) C_(12) C_(13) C_(14) C_(15) C_(16)
#undef C_
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_gather_box(const double *samples, int64_t n, int nz, int nr, double dz, double dr, int *box,
                             int *part, int max_blocks, hipStream_t s)
{
    if (n <= 0 || max_blocks <= 0) return hipErrorInvalidValue;
    const int64_t want = (n + 1023) / 1024;  // about four samples per thread
    const int blocks = (int)(want < max_blocks ? want : max_blocks);
    hipLaunchKernelGGL(k_gather_box, dim3((unsigned)blocks), dim3(256), 0, s, samples, n, nz, nr, dz, dr, part);
    hipLaunchKernelGGL(k_gather_box_reduce, dim3(1), dim3(256), 0, s, part, blocks, box);
    return hipGetLastError();
}

hipError_t launch_destagger(int prec, const DestaggerArgs &a, hipStream_t s)
{
    if (a.npass <= 0) return hipSuccess;
    const dim3 grid(512, (unsigned)a.npass);  // grid-stride over the box, one row of blocks per pass
    if (prec == P64) hipLaunchKernelGGL(k_destagger<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_destagger<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_gather(int prec, const GatherArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    if (a.ss != 0) {
        const dim3 grid((unsigned)((a.n + GATHER_BLOCK - 1) / GATHER_BLOCK));
#define FDETD_FINE(SS)                                                                                     \
    if (a.ss == SS) {                                                                                      \
        if (prec == P64) hipLaunchKernelGGL((k_gather_fine<double, SS>), grid, dim3(GATHER_BLOCK), 0, s, a); \
        else hipLaunchKernelGGL((k_gather_fine<float, SS>), grid, dim3(GATHER_BLOCK), 0, s, a);             \
    }
        FDETD_FINE(1) FDETD_FINE(2) FDETD_FINE(3)
#undef FDETD_FINE
        return hipGetLastError();
    }
    const dim3 grid((unsigned)((a.n + GATHER_BLOCK - 1) / GATHER_BLOCK));
    if (prec == P64) hipLaunchKernelGGL(k_gather<double>, grid, dim3(GATHER_BLOCK), 0, s, a);
    else hipLaunchKernelGGL(k_gather<float>, grid, dim3(GATHER_BLOCK), 0, s, a);
    return hipGetLastError();
}

// --------------------------------------------------------------------------------------------------
// Absorbing-layer damping (appendix on the scalar absorbing layer): both factors exp(-sigma dt/4) of the
// split step, applied to the cells where sigma = sigma_z + sigma_rho can be non-zero.  Thread t < lr nz
// takes row nr - lr + t / nz (the rho layer, every column); the others take the z layers of the rows
// above it, 2 lz cells per row.
// --------------------------------------------------------------------------------------------------
template <typename R>
__global__ __launch_bounds__(256) void k_absorb_damp(DampArgs A)
{
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long nrho = (long long)A.lr * A.nz, nzl = (long long)(A.nr - A.lr) * 2 * A.lz;
    if (t >= nrho + nzl) return;
    int k, i;
    if (t < nrho) {
        k = A.nr - A.lr + (int)(t / A.nz);
        i = (int)(t % A.nz);
    } else {
        const long long u = t - nrho;
        k = (int)(u / (2 * A.lz));
        const int c = (int)(u % (2 * A.lz));
        i = c < A.lz ? c : A.nz - 2 * A.lz + c;
    }
    const size_t q = (size_t)k * A.nz + i;
    const double d = exp(-(A.sz[i] + A.sr[k]) * A.qdt);
    if constexpr (std::is_same<R, double>::value) {
        double2 *a = (double2 *)A.a, *at = (double2 *)A.at;
        const double2 x = a[q], y = at[q];
        a[q] = double2{d * x.x, d * x.y};
        at[q] = double2{d * y.x, d * y.y};
    } else {
        float2 *a = (float2 *)A.a, *at = (float2 *)A.at;
        float2 *la = (float2 *)A.lo, *lt = la + (size_t)A.nz * A.nr;
        auto scale = [d](float &hi, float &lo) {
            const double x = d * ((double)hi + (double)lo);
            hi = (float)x;
            lo = (float)(x - (double)hi);
        };
        float2 x = a[q], y = at[q], lx = la[q], ly = lt[q];
        scale(x.x, lx.x);
        scale(x.y, lx.y);
        scale(y.x, ly.x);
        scale(y.y, ly.y);
        a[q] = x;
        at[q] = y;
        la[q] = lx;
        lt[q] = ly;
    }
}

hipError_t launch_absorb_damp(int prec, const DampArgs &a, hipStream_t s)
{
    const long long n = (long long)a.lr * a.nz + (long long)(a.nr - a.lr) * 2 * a.lz;
    if (n <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (prec == P64) hipLaunchKernelGGL(k_absorb_damp<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_absorb_damp<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_deposit_jz(int prec, const DepositArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t per_block = 256 * DEP_PER_THREAD;
    const dim3 g((unsigned)((a.n + per_block - 1) / per_block)), b(256);
    if (prec == P64) hipLaunchKernelGGL(k_deposit_jz<double>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_deposit_jz<float>, g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_deposit_current(int prec, const DepositArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t per_block = 256 * DEP_PER_THREAD;
    const dim3 grid((unsigned)((a.n + per_block - 1) / per_block));
    if (prec == P64) hipLaunchKernelGGL(k_deposit_current<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_deposit_current<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_deposit_rho(int prec, const DepositArgs &a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t per_block = 256 * DEP_PER_THREAD;
    const dim3 grid((unsigned)((a.n + per_block - 1) / per_block));
    if (prec == P64) hipLaunchKernelGGL(k_deposit_rho<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_deposit_rho<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_maxwell_stage(int prec, int nd, const MaxwellStageArgs &a, hipStream_t s)
{
    const dim3 g = tile_grid(a.nz, a.nr), b(TZ, TR, 1);
    return prec == P64 ? dispatch_nd<MaxwellL, double2>(nd, a, g, b, s)
                       : dispatch_nd<MaxwellL, float2>(nd, a, g, b, s);
}

hipError_t launch_envelope_stage(int prec, int nd, const EnvelopeStageArgs &a, hipStream_t s)
{
    const dim3 g = tile_grid(a.nz, a.nr), b(TZ, TR, 1);
    return prec == P64 ? dispatch_nd<EnvelopeL, double2>(nd, a, g, b, s)
                       : dispatch_nd<EnvelopeL, float2>(nd, a, g, b, s);
}

hipError_t launch_axis_fix_batch(int prec, const BatchArgs &a, int max_nz, hipStream_t s)
{
    const dim3 g((unsigned)((max_nz + 255) / 256), (unsigned)a.nprob), b(256, 1, 1);
    if (prec == P64) hipLaunchKernelGGL(k_axis_fix_batch<double2>, g, b, 0, s, a);
    else hipLaunchKernelGGL(k_axis_fix_batch<float2>, g, b, 0, s, a);
    return hipGetLastError();
}

hipError_t launch_axis_fix(int prec, int nd, const AxisArgs &a, hipStream_t s)
{
    const dim3 g((a.nz + 255) / 256, 1, 1), b(256, 1, 1);
    return prec == P64 ? dispatch_nd<AxisL, double2>(nd, a, g, b, s)
                       : dispatch_nd<AxisL, float2>(nd, a, g, b, s);
}

hipError_t launch_norm2(int prec, const void *x, size_t n, double *partial, int nblocks, hipStream_t s)
{
    if (prec == P64)
        hipLaunchKernelGGL(k_norm2<double2>, dim3(nblocks), dim3(256), 0, s, (const double2 *)x, n, partial);
    else
        hipLaunchKernelGGL(k_norm2<float2>, dim3(nblocks), dim3(256), 0, s, (const float2 *)x, n, partial);
    return hipGetLastError();
}

hipError_t launch_scale(int prec, void *x, size_t n, double alpha, hipStream_t s)
{
    const int nb = (int)((n + 255) / 256 < 4096 ? (n + 255) / 256 : 4096);
    if (prec == P64)
        hipLaunchKernelGGL(k_scale<double2>, dim3(nb), dim3(256), 0, s, (double2 *)x, n, alpha);
    else
        hipLaunchKernelGGL(k_scale<float2>, dim3(nb), dim3(256), 0, s, (float2 *)x, n, alpha);
    return hipGetLastError();
}

hipError_t launch_jgen(int prec, const JgenArgs &a, size_t max_cells, hipStream_t s)
{
    const size_t nb = (max_cells + 255) / 256;
    const dim3 g((unsigned)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096));
    if (prec == P64) hipLaunchKernelGGL(k_jgen<double2>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_jgen<float2>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_form_wn(int prec, const BatchArgs &a, size_t max_cells, hipStream_t s)
{
    const size_t nb = (max_cells + 255) / 256;
    const dim3 g((unsigned)(nb < 4096 ? (nb > 0 ? nb : 1) : 4096));
    if (prec == P64) hipLaunchKernelGGL(k_form_wn<double2>, g, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_form_wn<float2>, g, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy(const void *src, void *dst, size_t bytes, hipStream_t s)
{
    const size_t n = bytes / 8;
    const int nb = (int)((n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192);
    if (n) hipLaunchKernelGGL(k_copy8, dim3(nb > 0 ? nb : 1), dim3(256), 0, s, (const uint2 *)src, (uint2 *)dst, n);
    return hipGetLastError();
}

}  // namespace fdetd
