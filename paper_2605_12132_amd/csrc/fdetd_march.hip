// Row-marching gfx950 kernels of the FDETD Horner stage (Maxwell) and of the envelope stage.
//
// Layout of the work.  H_m = [[0, R], [-R, 0]] (section 2.1): the E part of H v reads only the B part of
// v and vice versa, so one Horner stage splits into two independent halves (E outputs from B inputs,
// B outputs from E inputs) that run as the two kinds of wavefront of one launch.  A wavefront owns a strip
// of consecutive z columns and marches down a segment of rho rows:
//   * FP64: lane pairs share a column (even lane: real part, odd lane: imaginary part), 32 columns per
//     wave; FP32: one lane per column holds the whole complex value, 64 columns per wave.  Either way a
//     row load of the strip is one coalesced 512-byte transaction and every stencil coefficient is real,
//     so lanes only meet for the i*m/rho terms (one lane swap in FP64);
//   * the two rho-stencilled inputs of its half live in a register window of 2 N_D rows that slides by
//     one row per step: each input row is loaded once per segment (section 2.3 staggered D^(+-) and
//     divergence D_div^(+-) along rho);
//   * the two z-stencilled inputs of the current row are staged in a per-wave LDS row with an N_D-column
//     halo on each side and read back at the 2 N_D tap offsets (section 2.3 D^(+-) along z);
//   * rows below the axis and the axis value (section 2.4) only occur while the window is first filled,
//     as wave-uniform branches.
// Tiles are numbered problem by problem and handed out so that each XCD (with its own L2) receives a
// contiguous range of them: neighbouring tiles, whose halos overlap, share an L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "fdetd_internal.h"
#include "fdetd_tiles.h"

namespace fdetd {
namespace {

constexpr int WAVE = 64;
constexpr int NXCD = 8;

// The share of one complex value a lane holds: one part (K = 1, FP64 lane pairs) or both (K = 2).
template <typename AR, int K>
struct lv {
    AR p[K];
};
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> operator+(lv<AR, K> a, lv<AR, K> b)
{
#pragma unroll
    for (int c = 0; c < K; ++c) a.p[c] += b.p[c];
    return a;
}
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> operator-(lv<AR, K> a, lv<AR, K> b)
{
#pragma unroll
    for (int c = 0; c < K; ++c) a.p[c] -= b.p[c];
    return a;
}
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> operator*(AR s, lv<AR, K> a)
{
#pragma unroll
    for (int c = 0; c < K; ++c) a.p[c] *= s;
    return a;
}
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> fmav(AR s, lv<AR, K> a, lv<AR, K> acc)
{
#pragma unroll
    for (int c = 0; c < K; ++c) acc.p[c] = fma(s, a.p[c], acc.p[c]);
    return acc;
}
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> zero_lv()
{
    lv<AR, K> z;
#pragma unroll
    for (int c = 0; c < K; ++c) z.p[c] = (AR)0;
    return z;
}
// i * s * x: (re, im) -> (-s im, s re); with lane pairs the partner lane holds the other part
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> times_i(AR s, lv<AR, K> x)
{
    lv<AR, K> r;
    if constexpr (K == 2) {
        r.p[0] = -s * x.p[1];
        r.p[1] = s * x.p[0];
    } else {
        const AR other = __shfl_xor(x.p[0], 1, WAVE);
        r.p[0] = (threadIdx.x & 1) ? s * other : -s * other;
    }
    return r;
}

// A coefficient of the Horner recurrence (dt/(n+1), the source weight -dt 2^-n) given in FP64 and applied
// to values in the arithmetic type AR.  Float arithmetic splits it, c = hi + lo with hi = float(c) and
// lo = float(c - hi), and forms c x as hi x + lo x: the product then carries c to about 2^-48 instead of
// rounding it to 2^-24, which would otherwise shift the effective time step the same way every stage.
template <typename AR>
struct Coef {
    AR hi, lo;
};
template <typename AR>
__device__ __forceinline__ Coef<AR> split_coef(double c)
{
    if constexpr (sizeof(AR) == 8) {
        return Coef<AR>{c, 0.0};
    } else {
        const float h = (float)c;
        return Coef<AR>{h, (float)(c - (double)h)};
    }
}
// c x
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> cmul(Coef<AR> c, lv<AR, K> x)
{
    if constexpr (sizeof(AR) == 8) return c.hi * x;
    else return fmav(c.lo, x, c.hi * x);
}
// c x + acc
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> cfma(Coef<AR> c, lv<AR, K> x, lv<AR, K> acc)
{
    if constexpr (sizeof(AR) == 8) return fmav(c.hi, x, acc);
    else return fmav(c.lo, x, fmav(c.hi, x, acc));
}

// FP32 storage read in lane pairs (one float part per lane, 32 columns per wave, as FP64 storage is read):
// the layout of the FP32C near-axis tiles, whose FP64 arithmetic on a whole complex value per lane would
// need twice the registers.
struct f2pair {};

template <typename V> struct scal;
template <> struct scal<double2> { using R = double; };
template <> struct scal<float2> { using R = float; };
template <> struct scal<f2pair> { using R = float; };
// storage element type of a layout (what pointers into the planes point at)
template <typename V> struct stor { using T = V; };
template <> struct stor<f2pair> { using T = float2; };

// Global-memory access through address-space-1 pointers.  The kernels' pointers come from a descriptor
// table and the kernel arguments, so without the cast the compiler emits flat instructions, which also
// count against the LDS/scalar wait counter and make every LDS wait drain the prefetched loads.
#define FDETD_GLOBAL __attribute__((address_space(1)))
template <typename T> struct ibits;  // an integer of the same size, to move T through global memory
template <> struct ibits<double> { using I = unsigned long long; };
template <> struct ibits<float2> { using I = unsigned long long; };
template <> struct ibits<float> { using I = unsigned int; };
// Element i of the array at p.  Callers pass a wave-uniform p (a row start, kept in scalar registers) and a
// small per-lane i, so the loads use the scalar-base + 32-bit-vector-offset addressing form.
// The byte offset is formed in 32 bits (a row of a plane is far below 4 GiB), which is what that addressing
// form adds to the scalar base.
// They go through a buffer resource whose base is that row start (four scalar registers built by scalar
// instructions) and take the lane's byte offset as the vector offset: no per-load vector address
// arithmetic.  Word 3 of the resource is the gfx9-family value for raw (untyped) buffer access; the
// record count is left at its maximum, every offset being a lane's position within its row.
constexpr int kBufWord3 = 0x00020000;
template <typename T>
__device__ __forceinline__ T gld(const void *p, unsigned i)
{
    using I = typename ibits<T>::I;
    const unsigned off = i * (unsigned)sizeof(I);
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, 0x7fffffff, kBufWord3);
    if constexpr (sizeof(I) == 8) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
template <typename T, int POL = 0>
__device__ __forceinline__ void gst(void *p, unsigned i, T v)
{
    using I = typename ibits<T>::I;
    const unsigned off = i * (unsigned)sizeof(I);
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(p, (short)0, 0x7fffffff, kBufWord3);
    if constexpr (sizeof(I) == 8) {
        using V2 = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0u, 0, 0));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(V2, v), r, off, 0, POL);
    } else {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, POL);
    }
}
// Store of a stage output: non-temporal (bit 1 of the cache-policy operand on this target family) in the
// kernel variants the plan picks when it measured them faster for a batch -- on grids far larger than the
// caches, outputs that the L2 keeps only evict the rows other wavefronts read again -- else the default.
template <typename T, bool NT>
__device__ __forceinline__ void gst_out(void *p, unsigned i, T v)
{
    gst<T, NT ? 2 : 0>(p, i, v);
}
// Start of row q of component c of a vector of planes of P elements each (row length nz S elements).
template <typename E>
__device__ __forceinline__ const E *row_ptr(const void *base, int c, size_t P, int nz, int S, int q)
{
    return (const E *)base + (size_t)c * P * S + (size_t)q * nz * S;
}
// The descriptor table and the per-row tables are written by the host before the launch and only read
// here: through the constant address space they become scalar loads the compiler may hoist, instead of
// vector loads whose in-order wait counter would also wait for the prefetched rows.
#define FDETD_CONST __attribute__((address_space(4)))
using CDesc = const FDETD_CONST ProbDesc;
__device__ __forceinline__ double cld(const double *p, int i) { return ((const FDETD_CONST double *)p)[i]; }
// Stencil coefficient j of a table in the arithmetic type: the float copy for float arithmetic (no
// conversion per tap), the double table otherwise.
template <typename AR>
__device__ __forceinline__ AR tap(const FDETD_CONST double *d, const FDETD_CONST float *f, int j)
{
    if constexpr (sizeof(AR) == 4) return f[j];
    else return d[j];
}

// Storage access.  FP64 (double2 storage, K = 1): element = one double, index 2*(row*nz + col) + part.
// FP32 (float2 storage, K = 2): element = one float2, index row*nz + col.
template <typename V> struct elem;
// Lo = the element of the FP32C compensation words in the same layout (unused with FP64 storage).
template <> struct elem<double2> {
    using E = double;
    using Lo = float2;
    static constexpr int S = 2;  // lanes per column
    static constexpr int K = 1;
};
template <> struct elem<float2> {
    using E = float2;
    using Lo = float2;
    static constexpr int S = 1;
    static constexpr int K = 2;
};
template <> struct elem<f2pair> {  // used only by the translation units of wide stencils
    using E = float;
    using Lo = float;
    [[maybe_unused]] static constexpr int S = 2;
    [[maybe_unused]] static constexpr int K = 1;
};

template <typename AR>
__device__ __forceinline__ lv<AR, 1> to_lv(double e) { return lv<AR, 1>{{(AR)e}}; }
template <typename AR>
__device__ __forceinline__ lv<AR, 2> to_lv(float2 e) { return lv<AR, 2>{{(AR)e.x, (AR)e.y}}; }
template <typename AR>
__device__ __forceinline__ lv<AR, 1> to_lv(float e) { return lv<AR, 1>{{(AR)e}}; }

__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// Wave-uniform facts of one tile of one problem in one stage.
struct Ctx {
    CDesc *D;
    const void *vin, *psi;
    void *vout;
    const void *jr, *jt, *jz;  // Jbar planes (null without source)
    const void *hi;            // increment form: the stored psi (hi words), read by the last stage
    int has_src, compensated;
    double beta_in, beta, coef;
};

// Lane geometry: column i = i0 + lane / S, element offset of (row 0, column i, part) = eidx.
template <typename V>
struct Lane {
    using T = elem<V>;
    int lane, i, eidx;
    bool col;
    __device__ Lane(int i0, int nz)
    {
        lane = threadIdx.x;
        i = i0 + lane / T::S;
        col = i < nz;
        const int ic = col ? i : nz - 1;  // clamped column: loads stay in bounds, values are masked
        eidx = ic * T::S + lane % T::S;
    }
};

// Element of row q of a plane for this lane.  A lane past the last grid column reads that column (clamped
// index): its results are never stored and never reach another lane, so the value needs no mask.
template <typename V>
__device__ __forceinline__ typename elem<V>::E ldraw(const typename stor<V>::T *plane, int nz, int q, const Lane<V> &L)
{
    using E = typename elem<V>::E;
    return gld<E>(row_ptr<E>(plane, 0, 0, nz, elem<V>::S, q), (unsigned)L.eidx);
}
template <typename V, typename AR>
__device__ __forceinline__ lv<AR, elem<V>::K> ldrow(const typename stor<V>::T *plane, int nz, int q, const Lane<V> &L)
{
    return to_lv<AR>(ldraw<V>(plane, nz, q, L));
}

// Store one output value: out = psi + inc (inc already holds beta*Jbar + coef*H v), or, in the last stage
// of an FP32C step, the exact TwoSum of (psi_hi, lo + inc) into (psi_hi, lo).  psi_v / lo_v are the values
// at the output position, loaded one row ahead.
template <typename V, typename AR, bool COMP, bool NT>
__device__ __forceinline__ void store_out(const Ctx &A, int c, int k, const Lane<V> &L, lv<AR, elem<V>::K> inc,
                                          bool zero_slot, typename elem<V>::E psi_v, typename elem<V>::Lo lo_v)
{
    using E = typename elem<V>::E;
    constexpr int S = elem<V>::S;
    CDesc &D = *A.D;
    void *orow = (void *)row_ptr<E>(A.vout, c, D.plane, D.nz, S, k);
    void *lrow = (void *)row_ptr<E>(D.lo, c, D.plane, D.nz, S, k);
    const unsigned o = (unsigned)L.eidx;
    if constexpr (S == 1) {
        if constexpr (COMP) {
            float sx, ex, sy, ey;
            two_sum(psi_v.x, (float)(inc.p[0] + (AR)lo_v.x), sx, ex);
            two_sum(psi_v.y, (float)(inc.p[1] + (AR)lo_v.y), sy, ey);
            if (zero_slot) sx = sy = ex = ey = 0.f;
            gst_out<float2, NT>(orow, o, float2{sx, sy});
            gst_out<float2, NT>(lrow, o, float2{ex, ey});
            return;
        }
        float2 w{(float)((AR)psi_v.x + inc.p[0]), (float)((AR)psi_v.y + inc.p[1])};
        if (zero_slot) w = float2{0.f, 0.f};
        gst_out<float2, NT>(orow, o, w);
    } else if constexpr (std::is_same<E, float>::value) {  // FP32 storage in lane pairs
        if constexpr (COMP) {
            float sx, ex;
            two_sum(psi_v, (float)(inc.p[0] + (AR)lo_v), sx, ex);
            if (zero_slot) sx = ex = 0.f;
            gst_out<float, NT>(orow, o, sx);
            gst_out<float, NT>(lrow, o, ex);
            return;
        }
        float w = (float)((AR)psi_v + inc.p[0]);
        if (zero_slot) w = 0.f;
        gst_out<float, NT>(orow, o, w);
    } else {
        double w = (double)((AR)psi_v + inc.p[0]);
        if (zero_slot) w = 0.0;
        gst_out<double, NT>(orow, o, w);
    }
}

// The E part of w_N = psi + beta_in Jbar (the argument of the highest power of H in the Horner form of
// the midpoint solution, section 2.1) for one loaded element: FP64 arithmetic, one rounding to the
// storage precision, the same operation as the separate w_N pass, so that both give the same bits.
__device__ __forceinline__ double wn_elem(double p, double j, double b) { return __builtin_fma(b, j, p); }
__device__ __forceinline__ float wn_elem(float p, float j, double b) { return (float)__builtin_fma(b, (double)j, (double)p); }
__device__ __forceinline__ float2 wn_elem(float2 p, float2 j, double b) { return float2{wn_elem(p.x, j.x, b), wn_elem(p.y, j.y, b)}; }
// Makes the value's computation happen here (an empty asm that takes and gives the value back).
__device__ __forceinline__ void pin(double &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(float &x) { asm volatile("" : "+v"(x)); }
__device__ __forceinline__ void pin(float2 &x)
{
    asm volatile("" : "+v"(x.x));
    asm volatile("" : "+v"(x.y));
}
// WN: the element of w_N from psi and Jbar; otherwise the loaded element itself.
template <bool WN, typename E>
__device__ __forceinline__ E wn_of(E p, E j, double b)
{
    if constexpr (WN) return wn_elem(p, j, b);
    else return p;
}

// The bracket coef multiplies: H v, or in the increment form P + H v (P = H psi of the step).
template <bool INC, typename AR, typename V>
__device__ __forceinline__ lv<AR, elem<V>::K> with_p(typename elem<V>::E p, lv<AR, elem<V>::K> hv)
{
    if constexpr (INC) return to_lv<AR>(p) + hv;
    else return hv;
}
// What store_out adds the increment to: psi (Horner on v), nothing (increment form, stages n > 0: the
// output is the increment itself), or the stored psi_hi (increment form, last stage, with lo).
template <bool INC, bool COMP, typename E>
__device__ __forceinline__ E out_base(E p, E h)
{
    if constexpr (!INC) return p;
    else if constexpr (COMP) return h;
    else return E{};
}

// Rows of input held in flight ahead of the row being computed.  One row of one wave is ~3 KB, and the
// launches have about two waves per SIMD, so HBM latency is covered only with several rows outstanding.
#ifndef FDETD_PREFETCH
#define FDETD_PREFETCH 4
#endif

// x if c, else +0.  The mask goes through an empty asm so that the compiler cannot see it is all-ones or
// zero: a select between a freshly loaded value and zero under a wave-uniform condition would otherwise
// become a branch around the load, and the wave would wait at its join for every load in flight.
template <typename AR, int K>
__device__ __forceinline__ lv<AR, K> keep_if(bool c, lv<AR, K> x)
{
    unsigned m = c ? ~0u : 0u;
    asm volatile("" : "+v"(m));
    lv<AR, K> r;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if constexpr (sizeof(AR) == 8) {
            const unsigned long long mm = ((unsigned long long)m << 32) | m;
            r.p[i] = __builtin_bit_cast(AR, __builtin_bit_cast(unsigned long long, x.p[i]) & mm);
        } else {
            r.p[i] = __builtin_bit_cast(AR, __builtin_bit_cast(unsigned, x.p[i]) & m);
        }
    }
    return r;
}

// March rows k0 .. k1-1: fill() loads the window of rows above k0, row(in, k, live) consumes the inputs of
// row k, fetch(k) issues the loads of row k.  PF rows are in flight, in a ring of PF slots; each slot is
// refilled in place once its row has been consumed: moving a slot whose loads are still in flight to
// another register would make the wave wait for them.  For the same reason a slot holds the loaded words
// only; masks, scale factors and sums are applied in row().  The loop body holds U rows (a multiple of PF):
// inside it the rho windows slide by renaming, and only at its end do they move between registers, so
// the moves per row fall as 1/U.  Rows past the segment end (fewer than U) run on the clamped last row
// with live = false and store nothing.
template <typename In, int PF, int U, typename Fetch, typename Row, typename Fill>
__device__ __forceinline__ void march_rows(int k0, int k1, Fetch &fetch, Row &row, Fill &fill)
{
    static_assert(U % PF == 0, "the loop body holds whole rounds of the ring");
    In ring[PF];
#pragma unroll
    for (int p = 0; p < PF; ++p) ring[p] = fetch(k0 + p < k1 ? k0 + p : k1 - 1);
    fill();
    // Drain the first loads before the loop: the wait counter is in-order, and a loop entered with the
    // ring's loads outstanding in another order than the loop issues them would have every row wait as if
    // for its slot being the newest.  (vmcnt 0; expcnt and lgkmcnt left at their maxima 7 and 15.)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int kb = k0; kb < k1; kb += U) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int k = kb + u;
            row(ring[u % PF], k < k1 ? k : k1 - 1, k < k1);
            const int kn = k + PF;
            ring[u % PF] = fetch(kn < k1 ? kn : k1 - 1);
        }
    }
}
// Rows per loop body of a code path: FDETD_ROW_UNROLL rounds of its prefetch ring.
#ifndef FDETD_ROW_UNROLL
#define FDETD_ROW_UNROLL 2
#endif

// Prefetch depth of a code path.  HEAVY paths (the first
// stage's current rows, the last stage's compensation words) carry more words per row and keep one row
// less.  Wider stencils hold a longer rho window (2 N_D rows) and keep fewer rows in flight.  The aim is two
// wavefronts per SIMD (at most 256 registers per lane).
template <typename V, typename AR, int ND, bool HEAVY>
constexpr int prefetch_of()
{
#ifdef FDETD_ANY_WIDTH
    // one kernel for every width has the registers of the widest, two wavefronts per SIMD whatever the ring
    constexpr int base = ND <= 8 ? FDETD_PREFETCH : (ND <= 12 ? FDETD_PREFETCH - 1 : FDETD_PREFETCH - 2);
#else
    // per width: two rows at N_D >= 9 (at 9 .. 12 3.4-4.8 % faster than three, partly from a third
    // wavefront per SIMD; one row at 13 .. 16 and three at <= 8 were slower)
    constexpr int base = ND <= 8 ? FDETD_PREFETCH : FDETD_PREFETCH - 2;
#endif
    // FP64 arithmetic on whole complex values per lane (near-axis tiles of narrow stencils): 2 rows
    constexpr bool wide = sizeof(AR) > sizeof(typename scal<V>::R) && elem<V>::K == 2;
    constexpr int pf = wide ? 2 : (HEAVY ? base - 1 : base);
    return pf < 1 ? 1 : pf;
}

// Raw element of (row q, this lane) of a 6-plane vector's component c, and the compensation word.
template <typename V>
__device__ __forceinline__ typename elem<V>::E ld_elem(const void *base, int c, int q, CDesc &D, const Lane<V> &L)
{
    using E = typename elem<V>::E;
    constexpr int S = elem<V>::S;
    return gld<E>(row_ptr<E>(base, c, D.plane, D.nz, S, q), (unsigned)L.eidx);
}

// One row of a plane as this lane contributes it to an LDS row with N_D columns of halo on each side:
// its own element and (lanes < 2 N_D S) one halo element.  Raw loads; put_row masks them.
template <typename V>
struct RowPart {
    typename elem<V>::E own, halo;
};
// Where this lane's halo element comes from and where it goes in the LDS row (fixed for a tile).
struct Halo {
    int slot;      // LDS slot
    unsigned idx;  // element index within a grid row (column 0 when outside the grid)
    bool ok;       // a halo lane whose column lies inside the grid
};
template <typename V, int ND>
__device__ __forceinline__ Halo halo_of(int i0, int nz, const Lane<V> &L)
{
    constexpr int S = elem<V>::S;
    Halo h;
    h.slot = L.lane < ND * S ? L.lane : WAVE + L.lane;
    const int ii = i0 - ND + h.slot / S;
    h.ok = L.lane < 2 * ND * S && ii >= 0 && ii < nz;
    h.idx = (unsigned)((h.ok ? ii : 0) * S + h.slot % S);
    return h;
}
template <typename V>
__device__ __forceinline__ RowPart<V> fetch_row(const typename stor<V>::T *plane, int nz, int q, const Lane<V> &L,
                                                const Halo &H)
{
    using E = typename elem<V>::E;
    constexpr int S = elem<V>::S;
    const E *prow = row_ptr<E>(plane, 0, 0, nz, S, q);
    RowPart<V> r;
    r.own = gld<E>(prow, (unsigned)L.eidx);
    r.halo = gld<E>(prow, H.idx);
    return r;
}
// The halo element of row q for this lane (the own element comes from a register window or an LDS ring).
template <typename V>
__device__ __forceinline__ typename elem<V>::E fetch_halo(const typename stor<V>::T *plane, int nz, int q, const Halo &H)
{
    using E = typename elem<V>::E;
    return gld<E>(row_ptr<E>(plane, 0, 0, nz, elem<V>::S, q), H.idx);
}
// A window value as the storage element it was loaded from (exact: an unscaled window of loaded values).
template <typename E, typename AR, int K>
__device__ __forceinline__ E from_lv(lv<AR, K> x)
{
    if constexpr (std::is_same<E, float2>::value) return float2{(float)x.p[0], (float)x.p[1]};
    else return (E)x.p[0];
}
// Columns outside the grid enter the z stencils as zeros.
template <typename V, int ND>
__device__ __forceinline__ void put_row(const RowPart<V> &r, const Lane<V> &L, const Halo &H, typename elem<V>::E *row)
{
    using E = typename elem<V>::E;
    constexpr int S = elem<V>::S;
    row[L.lane + ND * S] = L.col ? r.own : E{};
    if (L.lane < 2 * ND * S) row[H.slot] = H.ok ? r.halo : E{};
}

template <typename AR, typename V>
__device__ __forceinline__ lv<AR, elem<V>::K> lds_at(const typename elem<V>::E *row, int idx)
{
    return to_lv<AR>(row[idx]);
}

// --------------------------------------------------------------------------------------------------
// E half:  dE_rho   = -D_z^(+) B_theta + (i m / rho_(-)) B_z          (staggered rows k >= 1)
//          dE_theta =  D_z^(+) B_rho   - D_rho^(+,mS) B_z
//          dE_z     = -(i m / rho) B_rho + rho^-1 D^(+) (rho_(-) B_theta)
// Window (staggered rows q = k - N_D + 1 + t, t = 0 .. 2N_D-1): B_z and g = rho_(-) B_theta.
// --------------------------------------------------------------------------------------------------
template <typename V, typename AR, int ND, bool SRC, bool COMP, bool INC, bool NT>
__device__ __forceinline__ void e_half(const Ctx &A, int i0, int k0, int k1, typename elem<V>::E (*lds)[WAVE + 2 * ND * elem<V>::S])
{
    // ring of the last N_D + 1 raw B_theta rows (own elements): the z stencil of row k reads row k from here,
    // where it was put when it entered the rho window N_D rows earlier, instead of loading it again
    constexpr int RD = ND + 1;
    typename elem<V>::E *ring = &lds[2][0];
    constexpr int K = elem<V>::K, S = elem<V>::S;
    using L_ = lv<AR, K>;
    CDesc &D = *A.D;
    const int nz = D.nz, nr = D.nr;
    const Lane<V> L(i0, nz);
    const size_t P = D.plane;
    using SV = typename stor<V>::T;
    const SV *vin = (const SV *)A.vin;
    const SV *Bth = vin + BTH * P, *Br = vin + BR * P, *Bz = vin + BZ * P;
    const AR dr = (AR)D.dr, pS = (AR)D.pS, pA = -(AR)D.pS, mm = (AR)D.m;
    const L_ zero = zero_lv<AR, K>();

    L_ Wz[2 * ND], Wg[2 * ND];
    // filled after the ring's first loads are issued, so that both arrive within one latency
    auto fill = [&]() {
        L_ ax = zero;  // B_z on the axis: extrapolated for m = 0, else 0
        if (D.m == 0 && k0 < ND) {
#pragma unroll
            for (int q = 1; q <= ND; ++q) ax = fmav((AR)D.cax[q - 1], ldrow<V, AR>(Bz, nz, q, L), ax);
        }
        // staggered-grid window rows q = k0 - N_D + 1 + t: row 0 is the axis (B_z: ax; rho_(-) B_theta: 0),
        // rows q < 0 mirror row -q with the component's sign, rows >= nr are 0.  All loads are issued first
        // (clamped, valid rows), the rules are applied as selects afterwards.
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            const int q = k0 - ND + 1 + t;
            const int r = min(q < 0 ? -q : q, nr - 1);
            Wz[t] = ldrow<V, AR>(Bz, nz, r, L);
            Wg[t] = ldrow<V, AR>(Bth, nz, r, L);
        }
        // rows k0 .. k0 + N_D - 1 of B_theta, as loaded, for their z stencils
#pragma unroll
        for (int t = ND - 1; t < 2 * ND - 1; ++t) ring[((k0 - ND + 1 + t) % RD) * WAVE + L.lane] = from_lv<typename elem<V>::E>(Wg[t]);
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            const int q = k0 - ND + 1 + t;
            const AR sz = q < 0 ? pS : (AR)1, sg = q < 0 ? pA : (AR)1;
            Wz[t] = q >= nr ? zero : (q == 0 ? ax : sz * Wz[t]);
            Wg[t] = (q >= nr || q == 0) ? zero : ((AR)q * dr * sg) * Wg[t];
        }
    };
    const int own = L.lane + ND * S;
    using E = typename elem<V>::E;
    const Halo H = halo_of<V, ND>(i0, nz, L);
    // everything row k needs from memory: loads of valid rows only (indices clamped), formed in row()
    struct In {
        E bz, bt, j0, j1, j2, thh;
        RowPart<V> br;
        E p0, p1, p2;
        typename elem<V>::Lo l0, l1, l2;
        E h0, h1, h2;
    };
    auto fetch = [&](int k) -> In {
        In x;
        const int qn = k + ND;
        const int qc = qn < nr ? qn : nr - 1;
        x.bz = ldraw<V>(Bz, nz, qc, L);
        x.bt = ldraw<V>(Bth, nz, qc, L);
        x.thh = fetch_halo<V>(Bth, nz, k, H);
        x.br = fetch_row<V>(Br, nz, k, L, H);
        x.j0 = x.j1 = x.j2 = E{};
        if constexpr (SRC) {
            x.j0 = ldraw<V>((const SV *)A.jr, nz, k, L);
            x.j1 = ldraw<V>((const SV *)A.jt, nz, k, L);
            x.j2 = ldraw<V>((const SV *)A.jz, nz, k, L);
        }
        x.p0 = ld_elem<V>(A.psi, ER, k, D, L);
        x.p1 = ld_elem<V>(A.psi, ETH, k, D, L);
        x.p2 = ld_elem<V>(A.psi, EZ, k, D, L);
        x.l0 = x.l1 = x.l2 = typename elem<V>::Lo{};
        if constexpr (COMP) {
            x.l0 = ld_elem<V>(D.lo, ER, k, D, L);
            x.l1 = ld_elem<V>(D.lo, ETH, k, D, L);
            x.l2 = ld_elem<V>(D.lo, EZ, k, D, L);
        }
        x.h0 = x.h1 = x.h2 = E{};
        if constexpr (INC && COMP) {
            x.h0 = ld_elem<V>(A.hi, ER, k, D, L);
            x.h1 = ld_elem<V>(A.hi, ETH, k, D, L);
            x.h2 = ld_elem<V>(A.hi, EZ, k, D, L);
        }
        return x;
    };
    auto row = [&](const In &cu, int k, bool live) {
        const int qn = k + ND;  // the window's new row
        Wz[2 * ND - 1] = keep_if(qn < nr, to_lv<AR>(cu.bz));
        Wg[2 * ND - 1] = keep_if(qn < nr, ((AR)qn * dr) * to_lv<AR>(cu.bt));
        ring[(qn % RD) * WAVE + L.lane] = cu.bt;
        put_row<V, ND>(RowPart<V>{ring[(k % RD) * WAVE + L.lane], cu.thh}, L, H, lds[0]);
        put_row<V, ND>(cu.br, L, H, lds[1]);
        __syncthreads();
        L_ zth = zero, zr = zero, rz = zero, rg = zero;
        // D_z^(+) at primary column i: staggered columns i + j and i - j + 1
#pragma unroll 4
        for (int j = 1; j <= ND; ++j) {
            const AR az = tap<AR>(D.az, D.azf, j - 1);
            zth = fmav(az, lds_at<AR, V>(lds[0], own + j * S) - lds_at<AR, V>(lds[0], own - (j - 1) * S), zth);
            zr = fmav(az, lds_at<AR, V>(lds[1], own + j * S) - lds_at<AR, V>(lds[1], own - (j - 1) * S), zr);
        }
        // D^(+) along rho at primary row k: staggered rows k + j (slot ND-1+j) and k - j + 1 (slot ND-j)
#pragma unroll
        for (int j = 1; j <= ND; ++j) {
            const AR ar = tap<AR>(D.ar, D.arf, j - 1);
            rz = fmav(ar, Wz[ND - 1 + j] - Wz[ND - j], rz);
            rg = fmav(ar, Wg[ND - 1 + j] - Wg[ND - j], rg);
        }
        const L_ br = to_lv<AR>(cu.br.own);
        const L_ bzk = Wz[ND - 1];
        const AR rip = (AR)cld(D.rinv_p, k), ris = (AR)cld(D.rinv_s, k);
        const L_ t0 = times_i(mm * ris, bzk);  // lane swaps: every lane of the wave takes part
        const L_ t2 = times_i(mm * rip, br);
        __syncthreads();
        if (L.col && live) {
            const Coef<AR> coef = split_coef<AR>(A.coef), beta = split_coef<AR>(A.beta);
            const L_ i0v = cfma(beta, to_lv<AR>(cu.j0), cmul(coef, with_p<INC, AR, V>(cu.p0, t0 - zth)));
            const L_ i1v = cfma(beta, to_lv<AR>(cu.j1), cmul(coef, with_p<INC, AR, V>(cu.p1, zr - rz)));
            const L_ i2v = cfma(beta, to_lv<AR>(cu.j2), cmul(coef, with_p<INC, AR, V>(cu.p2, rip * rg - t2)));
            store_out<V, AR, COMP, NT>(A, ER, k, L, i0v, k == 0, out_base<INC, COMP>(cu.p0, cu.h0), cu.l0);
            store_out<V, AR, COMP, NT>(A, ETH, k, L, i1v, false, out_base<INC, COMP>(cu.p1, cu.h1), cu.l1);
            store_out<V, AR, COMP, NT>(A, EZ, k, L, i2v, false, out_base<INC, COMP>(cu.p2, cu.h2), cu.l2);
        }
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            Wz[t] = Wz[t + 1];
            Wg[t] = Wg[t + 1];
        }
    };
    march_rows<In, prefetch_of<V, AR, ND, COMP>(), FDETD_ROW_UNROLL * prefetch_of<V, AR, ND, COMP>()>(k0, k1, fetch, row, fill);
}

// --------------------------------------------------------------------------------------------------
// B half:  dB_rho   =  D_z^(-) E_theta - (i m / rho) E_z
//          dB_theta = -D_z^(-) E_rho   + D_rho^(-,mS) E_z              (staggered rows k >= 1)
//          dB_z     =  (i m / rho_(-)) E_rho - rho_(-)^-1 D^(-) (rho E_theta)   (k >= 1)
// Window (primary rows q = k - N_D + t, t = 0 .. 2N_D-1): E_z and g = rho E_theta.
// In the first stage of a step with a current the E input is w_N = psi + beta_in Jbar, formed as psi and
// Jbar are loaded (WN) or, where the plan forms it in a pass of its own (k_form_wn), read from that pass's
// plane; otherwise psi or the previous stage's output.
// --------------------------------------------------------------------------------------------------
// WN: the first stage of a step with a current, whose input E part is w_N = psi + beta_in Jbar: vin is psi
// and each loaded E element is combined with the Jbar element at the same place as it arrives, instead of
// being read from a w_N plane formed by a separate pass.
template <typename V, typename AR, int ND, bool COMP, bool INC, bool WN, bool NT>
__device__ __forceinline__ void b_half(const Ctx &A, int i0, int k0, int k1, typename elem<V>::E (*lds)[WAVE + 2 * ND * elem<V>::S])
{
    // ring of the last N_D + 1 raw E_theta rows (own elements), as in e_half
    constexpr int RD = ND + 1;
    typename elem<V>::E *ring = &lds[2][0];
    constexpr int K = elem<V>::K, S = elem<V>::S;
    using L_ = lv<AR, K>;
    CDesc &D = *A.D;
    const int nz = D.nz, nr = D.nr;
    const Lane<V> L(i0, nz);
    const size_t P = D.plane;
    using SV = typename stor<V>::T;
    const SV *vin = (const SV *)A.vin;
    const SV *Er = vin + ER * P, *Eth = vin + ETH * P, *Ez = vin + EZ * P;
    const SV *Jr = (const SV *)A.jr, *Jt = (const SV *)A.jt, *Jz = (const SV *)A.jz;  // WN only
    const double bw = A.beta_in;
    const AR dr = (AR)D.dr, pS = (AR)D.pS, pA = -(AR)D.pS, mm = (AR)D.m;
    const L_ zero = zero_lv<AR, K>();
    L_ Wz[2 * ND], Wg[2 * ND];
    // filled after the ring's first loads are issued, so that both arrive within one latency
    auto fill = [&]() {
        // primary-grid window rows q = k0 - N_D + t: rows q < 0 mirror row -1-q with the component's sign,
        // rows >= nr are 0; loads first (clamped rows), rules as selects.
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            const int q = k0 - ND + t;
            const int r = min(q < 0 ? -1 - q : q, nr - 1);
            if constexpr (WN) {
                // each sum formed (pinned) as its row arrives: otherwise the compiler sinks every sum to
                // the end of the fill, and the psi and Jbar elements of all 2 N_D - 1 rows are held in
                // registers at once beside the window (two wavefronts per SIMD would no longer fit)
                typename elem<V>::E wz = wn_elem(ldraw<V>(Ez, nz, r, L), ldraw<V>(Jz, nz, r, L), bw);
                typename elem<V>::E wt = wn_elem(ldraw<V>(Eth, nz, r, L), ldraw<V>(Jt, nz, r, L), bw);
                pin(wz);
                pin(wt);
                Wz[t] = to_lv<AR>(wz);
                Wg[t] = to_lv<AR>(wt);
            } else {
                Wz[t] = ldrow<V, AR>(Ez, nz, r, L);
                Wg[t] = ldrow<V, AR>(Eth, nz, r, L);
            }
        }
        // rows k0 .. k0 + N_D - 2 of E_theta, as loaded, for their z stencils
#pragma unroll
        for (int t = ND; t < 2 * ND - 1; ++t) ring[((k0 - ND + t) % RD) * WAVE + L.lane] = from_lv<typename elem<V>::E>(Wg[t]);
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            const int q = k0 - ND + t;
            const AR sz = q < 0 ? pS : (AR)1, sg = q < 0 ? pA : (AR)1;
            Wz[t] = q >= nr ? zero : sz * Wz[t];
            Wg[t] = q >= nr ? zero : ((((AR)q + (AR)0.5) * dr) * sg) * Wg[t];
        }
    };
    const int own = L.lane + ND * S;
    using E = typename elem<V>::E;
    const Halo H = halo_of<V, ND>(i0, nz, L);
    struct In {
        E ez, et, thh;
        RowPart<V> er;
        E jez, jet, jthh;  // WN: the Jbar elements at the same places
        RowPart<V> jer;
        E p0, p1, p2;
        typename elem<V>::Lo l0, l1, l2;
        E h0, h1, h2;
    };
    auto fetch = [&](int k) -> In {
        In x;
        const int qn = k + ND - 1;
        const int qc = qn < nr ? qn : nr - 1;
        x.ez = ldraw<V>(Ez, nz, qc, L);
        x.et = ldraw<V>(Eth, nz, qc, L);
        x.thh = fetch_halo<V>(Eth, nz, k, H);
        x.er = fetch_row<V>(Er, nz, k, L, H);
        x.jez = x.jet = x.jthh = E{};
        x.jer = RowPart<V>{E{}, E{}};
        if constexpr (WN) {
            x.jez = ldraw<V>(Jz, nz, qc, L);
            x.jet = ldraw<V>(Jt, nz, qc, L);
            x.jthh = fetch_halo<V>(Jt, nz, k, H);
            x.jer = fetch_row<V>(Jr, nz, k, L, H);
        }
        x.p0 = ld_elem<V>(A.psi, BR, k, D, L);
        x.p1 = ld_elem<V>(A.psi, BTH, k, D, L);
        x.p2 = ld_elem<V>(A.psi, BZ, k, D, L);
        x.l0 = x.l1 = x.l2 = typename elem<V>::Lo{};
        if constexpr (COMP) {
            x.l0 = ld_elem<V>(D.lo, BR, k, D, L);
            x.l1 = ld_elem<V>(D.lo, BTH, k, D, L);
            x.l2 = ld_elem<V>(D.lo, BZ, k, D, L);
        }
        x.h0 = x.h1 = x.h2 = E{};
        if constexpr (INC && COMP) {
            x.h0 = ld_elem<V>(A.hi, BR, k, D, L);
            x.h1 = ld_elem<V>(A.hi, BTH, k, D, L);
            x.h2 = ld_elem<V>(A.hi, BZ, k, D, L);
        }
        return x;
    };
    auto row = [&](const In &cu, int k, bool live) {
        const int qn = k + ND - 1;  // the window's new row
        const E etw = wn_of<WN>(cu.et, cu.jet, bw);
        const RowPart<V> erw{wn_of<WN>(cu.er.own, cu.jer.own, bw), wn_of<WN>(cu.er.halo, cu.jer.halo, bw)};
        const L_ ez = to_lv<AR>(wn_of<WN>(cu.ez, cu.jez, bw)), et = to_lv<AR>(etw);
        Wz[2 * ND - 1] = keep_if(qn < nr, ez);
        Wg[2 * ND - 1] = keep_if(qn < nr, (((AR)qn + (AR)0.5) * dr) * et);
        ring[(qn % RD) * WAVE + L.lane] = etw;
        put_row<V, ND>(RowPart<V>{ring[(k % RD) * WAVE + L.lane], wn_of<WN>(cu.thh, cu.jthh, bw)}, L, H, lds[0]);
        put_row<V, ND>(erw, L, H, lds[1]);
        __syncthreads();
        L_ zth = zero, zr = zero, rz = zero, rg = zero;
        // D_z^(-) at staggered column i: primary columns i + j - 1 and i - j
#pragma unroll 4
        for (int j = 1; j <= ND; ++j) {
            const AR az = tap<AR>(D.az, D.azf, j - 1);
            zth = fmav(az, lds_at<AR, V>(lds[0], own + (j - 1) * S) - lds_at<AR, V>(lds[0], own - j * S), zth);
            zr = fmav(az, lds_at<AR, V>(lds[1], own + (j - 1) * S) - lds_at<AR, V>(lds[1], own - j * S), zr);
        }
        // D^(-) along rho at staggered row k: primary rows k + j - 1 (slot ND+j-1) and k - j (slot ND-j)
#pragma unroll
        for (int j = 1; j <= ND; ++j) {
            const AR ar = tap<AR>(D.ar, D.arf, j - 1);
            rz = fmav(ar, Wz[ND + j - 1] - Wz[ND - j], rz);
            rg = fmav(ar, Wg[ND + j - 1] - Wg[ND - j], rg);
        }
        const L_ erk = to_lv<AR>(erw.own);
        const L_ ezk = Wz[ND];
        const AR rip = (AR)cld(D.rinv_p, k), ris = (AR)cld(D.rinv_s, k);
        const L_ t0 = times_i(mm * rip, ezk);
        const L_ t2 = times_i(mm * ris, erk);
        __syncthreads();
        if (L.col && live) {
            const Coef<AR> coef = split_coef<AR>(A.coef);
            store_out<V, AR, COMP, NT>(A, BR, k, L, cmul(coef, with_p<INC, AR, V>(cu.p0, zth - t0)), false,
                                   out_base<INC, COMP>(cu.p0, cu.h0), cu.l0);
            store_out<V, AR, COMP, NT>(A, BTH, k, L, cmul(coef, with_p<INC, AR, V>(cu.p1, rz - zr)), k == 0,
                                   out_base<INC, COMP>(cu.p1, cu.h1), cu.l1);
            store_out<V, AR, COMP, NT>(A, BZ, k, L, cmul(coef, with_p<INC, AR, V>(cu.p2, t2 - ris * rg)), k == 0,
                                   out_base<INC, COMP>(cu.p2, cu.h2), cu.l2);
        }
#pragma unroll
        for (int t = 0; t < 2 * ND - 1; ++t) {
            Wz[t] = Wz[t + 1];
            Wg[t] = Wg[t + 1];
        }
    };
    constexpr int PF = prefetch_of<V, AR, ND, COMP>();
    march_rows<In, PF, FDETD_ROW_UNROLL * PF>(k0, k1, fetch, row, fill);
}

// Tile of block b.  Tiles are numbered problem by problem, (half,) segment, strip -- strips fastest --
// separately for the near-axis tiles (FP32 storage only) and the main tiles.  XCD x (the blocks with
// b % 8 == x) first receives the near-axis range [x * per_ax, (x + 1) * per_ax), then the main range
// [x * per, (x + 1) * per): every XCD (with its own L2) gets neighbouring tiles, and the slower near-axis
// tiles are dispatched first and spread over all XCDs.  Returns -1 past the end of either range.
__device__ __forceinline__ int tile_of_block(int ntiles_ax, int ntiles, bool &axis)
{
    const int per_ax = (ntiles_ax + NXCD - 1) / NXCD, per = (ntiles + NXCD - 1) / NXCD;
    const int x = (int)(blockIdx.x % NXCD), slot = (int)(blockIdx.x / NXCD);
    axis = slot < per_ax;
    const int t = axis ? x * per_ax + slot : x * per + (slot - per_ax);
    return t < (axis ? ntiles_ax : ntiles) ? t : -1;
}
// Blocks of a launch: NXCD * (per_ax + per).
inline int blocks_of(int ntiles_ax, int ntiles)
{
    return NXCD * ((ntiles_ax + NXCD - 1) / NXCD + (ntiles + NXCD - 1) / NXCD);
}

template <bool AXIS>
__device__ __forceinline__ int problem_of_tile(const BatchArgs &A, int t)
{
    CDesc *T = (CDesc *)A.probs;
    int p = 0;
    while (p + 1 < A.nprob && (AXIS ? T[p + 1].tile_begin_ax : T[p + 1].tile_begin) <= t) ++p;
    return p;
}

// AXIS = false: rows ax_rows .. nr-1 in the storage precision; AXIS = true (FP32 storage; V = float2 or,
// for wide stencils, f2pair read in lane pairs): rows 0 .. ax_rows-1 (= 2 N_D), whose stencils reach the
// axis and its 1/rho factors, in FP64 arithmetic.
template <typename V, int ND, bool SRC, bool COMP, bool INC, bool AXIS, bool WN, bool NT>
__device__ __forceinline__ void maxwell_tile(const BatchArgs &A, int t, typename elem<V>::E (*lds)[WAVE + 2 * ND * elem<V>::S])
{
    constexpr int S = elem<V>::S, CPW = WAVE / S;
    const int p = problem_of_tile<AXIS>(A, t);
    CDesc &D = ((CDesc *)A.probs)[p];
    TileCoord tc;
    if (!decode_tile(D, t - (AXIS ? D.tile_begin_ax : D.tile_begin), 2, AXIS, CPW, tc)) return;
    const int half = tc.half, i0 = tc.i0, k0 = tc.k0, k1 = tc.k1;
    Ctx C;
    C.D = &D;
    const bool first = A.n == A.N - 1;
    if constexpr (INC) {
        // increment form: the psi slot holds P.  Role 1: P = H lo (from the zero planes); role 2: P += H
        // psi_hi, in place (P is read only at the output position).  Stages: vin = d_{n+1}; the first
        // stage's d_N is beta_in Jbar in its E part (k_form_wn, second stage buffer) and zero in its B
        // part; the last stage adds d_0 into (psi_hi, lo) in place.
        if (A.role == 1) {
            C.vin = D.lo;
            C.psi = D.zero;
            C.vout = D.pbuf;
        } else if (A.role == 2) {
            C.vin = A.psi[p];
            C.psi = D.pbuf;
            C.vout = D.pbuf;
        } else {
            C.vin = first ? ((A.has_src && half == 1) ? D.buf[1] : D.zero) : D.buf[(A.N - 2 - A.n) & 1];
            C.psi = D.pbuf;
            C.vout = A.n == 0 ? (void *)A.psi[p] : D.buf[(A.N - 1 - A.n) & 1];
        }
        C.hi = A.psi[p];
    } else {
        C.psi = A.psi[p];
        // the first stage reads psi, except the B half of a step with a current: it reads the E part of
        // w_N = psi + beta_in Jbar, which k_form_wn wrote into the second stage buffer before the launch,
        // or (WN) forms it from psi and Jbar as it loads them
        C.vin = first ? ((A.has_src && half == 1 && !WN) ? D.buf[1] : C.psi) : D.buf[(A.N - 2 - A.n) & 1];
        C.vout = (A.n == 0 && A.N > 1) ? (void *)C.psi : D.buf[(A.N - 1 - A.n) & 1];
        C.hi = nullptr;
    }
    C.has_src = A.has_src;
    const size_t pb = D.plane * sizeof(typename stor<V>::T);
    C.jr = A.has_src ? D.jbar : nullptr;
    C.jt = A.has_src ? (D.jth ? D.jth : (const char *)A.aux[p] + pb) : nullptr;  // corrected J_theta if any
    C.jz = A.has_src ? (const char *)A.aux[p] + 2 * pb : nullptr;
    C.compensated = A.compensated && A.n == 0 && A.role == 0;
    C.beta_in = A.beta_in;
    C.beta = A.beta;
    C.coef = A.coef;
    using AR = typename std::conditional<AXIS, double, typename scal<V>::R>::type;
    if (half == 0) e_half<V, AR, ND, SRC, COMP, INC, NT>(C, i0, k0, k1, lds);
    else b_half<V, AR, ND, COMP, INC, WN, NT>(C, i0, k0, k1, lds);
}

// One Horner stage of every problem of a batch, near-axis and main tiles in one launch.
// Bytes of one LDS row of a layout.
template <typename V, int ND>
constexpr int lds_row_bytes()
{
    return (WAVE + 2 * ND * elem<V>::S) * (int)sizeof(typename elem<V>::E);
}
constexpr int cmax(int a, int b) { return a > b ? a : b; }
// LDS of one stage wavefront: the two z-stencil rows, then N_D + 1 rows of own elements (the theta ring)
template <typename V, int ND>
constexpr int stage_lds_bytes()
{
    return 2 * lds_row_bytes<V, ND>() + (ND + 1) * WAVE * (int)sizeof(typename elem<V>::E);
}

template <typename V, int ND, bool SRC, bool COMP, bool INC, bool WN, bool NT>
__global__ __launch_bounds__(WAVE) void k_maxwell_stage(BatchArgs A)
{
    // layout of the near-axis tiles (FP32 storage only): whole complex values per lane or lane pairs
    using VA = typename std::conditional<(ND <= kAxisWholeND), float2, f2pair>::type;
    // two LDS rows and the ring of raw theta rows, sized for the main layout and the near-axis one
    __shared__ __align__(16) unsigned char smem[cmax(stage_lds_bytes<V, ND>(), stage_lds_bytes<VA, ND>())];
    bool axis;
    const int t = tile_of_block(A.ntiles_ax, A.ntiles, axis);
    if (t < 0) return;
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if (axis) {
            using EA = typename elem<VA>::E;
            maxwell_tile<VA, ND, SRC, COMP, INC, true, WN, NT>(A, t, (EA(*)[WAVE + 2 * ND * elem<VA>::S])smem);
            return;
        }
    }
    using E = typename elem<V>::E;
    maxwell_tile<V, ND, SRC, COMP, INC, false, WN, NT>(A, t, (E(*)[WAVE + 2 * ND * elem<V>::S])smem);
}

// --------------------------------------------------------------------------------------------------
// Envelope stage (section 4.2): out = psi + coef * H_a vin with
//   H_a (a, a~) = (a~, (L_rho + L_z - m^2/rho^2 - chi) a + 2 i k0 (D_z^(C) a + a~)),
// window of a over primary rows k - N_D .. k + N_D (scalar-like extension), current row of a in LDS.
// --------------------------------------------------------------------------------------------------
struct EnvCtx {
    CDesc *D;
    const void *vin_a, *vin_t, *psi_a, *psi_t, *chi;
    const void *hi_a, *hi_t;  // increment form: the stored a, a~ (hi words), read by the last stage
    void *out_a, *out_t;
    int compensated;
    double coef;
};

template <typename V, typename AR, int ND, bool COMP, bool INC>
__device__ __forceinline__ void env_march(const EnvCtx &A, int i0, int k0, int k1, typename elem<V>::E *lds)
{
    constexpr int K = elem<V>::K, S = elem<V>::S;
    using E = typename elem<V>::E;
    using R = typename scal<V>::R;
    using L_ = lv<AR, K>;
    CDesc &D = *A.D;
    const int nz = D.nz, nr = D.nr;
    const Lane<V> L(i0, nz);
    using SV = typename stor<V>::T;
    const SV *va = (const SV *)A.vin_a, *vt = (const SV *)A.vin_t;
    const L_ zero = zero_lv<AR, K>();
    const AR pS = (AR)D.pS;
    constexpr int W = 2 * ND + 1;
    L_ Wa[W];
    // filled after the ring's first loads are issued, so that both arrive within one latency
    auto fill = [&]() {
#pragma unroll
        for (int t = 0; t < W - 1; ++t) {
            const int q = k0 - ND + t;
            Wa[t] = ldrow<V, AR>(va, nz, min(q < 0 ? -1 - q : q, nr - 1), L);
        }
#pragma unroll
        for (int t = 0; t < W - 1; ++t) {
            const int q = k0 - ND + t;
            Wa[t] = q >= nr ? zero : (q < 0 ? pS : (AR)1) * Wa[t];
        }
    };
    const AR k2 = (AR)(2.0 * D.k0);
    const int own = L.lane + ND * S;
    const int cc = L.col ? L.i : nz - 1;
    const AR szi = (AR)gld<double>(D.sz, (unsigned)cc);  // absorbing layer: sigma_z of this column
    const Halo H = halo_of<V, ND>(i0, nz, L);
    struct In {
        E an, tin, ah;
        R chi;
        E pa, pt;
        typename elem<V>::Lo la, lt;
        E ha, ht;
    };
    auto fetch = [&](int k) -> In {
        In x;
        const int qn = k + ND;
        x.an = ldraw<V>(va, nz, qn < nr ? qn : nr - 1, L);
        x.ah = fetch_halo<V>(va, nz, k, H);
        x.tin = ldraw<V>(vt, nz, k, L);
        x.chi = gld<R>((const R *)A.chi + (size_t)k * nz, (unsigned)cc);
        const unsigned o = (unsigned)L.eidx;
        x.pa = gld<E>(row_ptr<E>(A.psi_a, 0, 0, nz, S, k), o);
        x.pt = gld<E>(row_ptr<E>(A.psi_t, 0, 0, nz, S, k), o);
        x.la = x.lt = typename elem<V>::Lo{};
        if constexpr (COMP) {
            using Lo = typename elem<V>::Lo;
            x.la = gld<Lo>(row_ptr<Lo>(D.lo, 0, D.plane, nz, S, k), o);
            x.lt = gld<Lo>(row_ptr<Lo>(D.lo, 1, D.plane, nz, S, k), o);
        }
        x.ha = x.ht = E{};
        if constexpr (INC && COMP) {
            x.ha = gld<E>(row_ptr<E>(A.hi_a, 0, 0, nz, S, k), o);
            x.ht = gld<E>(row_ptr<E>(A.hi_t, 0, 0, nz, S, k), o);
        }
        return x;
    };
    auto row = [&](const In &cu, int k, bool live) {
        const int qn = k + ND;
        Wa[W - 1] = keep_if(qn < nr, to_lv<AR>(cu.an));
        const L_ tin = to_lv<AR>(cu.tin);
        put_row<V, ND>(RowPart<V>{from_lv<E>(Wa[ND]), cu.ah}, L, H, lds);  // own element: the window's row k
        __syncthreads();
        const L_ a0 = Wa[ND];
        L_ lz = tap<AR>(D.bz, D.bzf, 0) * a0, d1z = zero;
#pragma unroll 4
        for (int j = 1; j <= ND; ++j) {
            const L_ zp = lds_at<AR, V>(lds, own + j * S), zm = lds_at<AR, V>(lds, own - j * S);
            lz = fmav(tap<AR>(D.bz, D.bzf, j), zp + zm, lz);
            d1z = fmav(tap<AR>(D.dzc, D.dzcf, j - 1), zp - zm, d1z);
        }
        L_ lr = tap<AR>(D.br, D.brf, 0) * a0, d1r = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) {
            const L_ rp = Wa[ND + j], rm = Wa[ND - j];
            lr = fmav(tap<AR>(D.br, D.brf, j), rp + rm, lr);
            d1r = fmav(tap<AR>(D.drc, D.drcf, j - 1), rp - rm, d1r);
        }
        // m^2 / rho^2 + chi~ with chi~ = chi + sigma^2 (absorbing layer; sigma = 0 outside it)
        const AR sig = szi + (AR)cld(D.sr, k);
        const AR pot = fma(sig, sig, (AR)cld(D.m2rinv2, k) + (AR)cu.chi);
        const L_ rot = times_i(k2, d1z + tin);
        __syncthreads();
        if (L.col && live) {
            const L_ dtv = lr + (AR)cld(D.rinv_p, k) * d1r + lz - pot * a0 + rot;
            const Coef<AR> coef = split_coef<AR>(A.coef);
            const L_ ia = cmul(coef, with_p<INC, AR, V>(cu.pa, tin)), it = cmul(coef, with_p<INC, AR, V>(cu.pt, dtv));
            // what the increment is added to: psi, nothing (increment form, n > 0) or the stored psi_hi
            const E ba = out_base<INC, COMP>(cu.pa, cu.ha), bt = out_base<INC, COMP>(cu.pt, cu.ht);
            const unsigned o = (unsigned)L.eidx;
            void *ra = (void *)row_ptr<E>(A.out_a, 0, 0, nz, S, k), *rt = (void *)row_ptr<E>(A.out_t, 0, 0, nz, S, k);
            if constexpr (S == 1) {
                if constexpr (COMP) {
                    float s0, e0, s1, e1, s2, e2, s3, e3;
                    two_sum(ba.x, (float)(ia.p[0] + (AR)cu.la.x), s0, e0);
                    two_sum(ba.y, (float)(ia.p[1] + (AR)cu.la.y), s1, e1);
                    two_sum(bt.x, (float)(it.p[0] + (AR)cu.lt.x), s2, e2);
                    two_sum(bt.y, (float)(it.p[1] + (AR)cu.lt.y), s3, e3);
                    gst<float2>(ra, o, float2{s0, s1});
                    gst<float2>(rt, o, float2{s2, s3});
                    gst<float2>((void *)row_ptr<float2>(D.lo, 0, D.plane, nz, 1, k), o, float2{e0, e1});
                    gst<float2>((void *)row_ptr<float2>(D.lo, 1, D.plane, nz, 1, k), o, float2{e2, e3});
                } else {
                    gst<float2>(ra, o, float2{(float)((AR)ba.x + ia.p[0]), (float)((AR)ba.y + ia.p[1])});
                    gst<float2>(rt, o, float2{(float)((AR)bt.x + it.p[0]), (float)((AR)bt.y + it.p[1])});
                }
            } else if constexpr (std::is_same<E, float>::value) {  // FP32 storage in lane pairs
                if constexpr (COMP) {
                    float s0, e0, s1, e1;
                    two_sum(ba, (float)(ia.p[0] + (AR)cu.la), s0, e0);
                    two_sum(bt, (float)(it.p[0] + (AR)cu.lt), s1, e1);
                    gst<float>(ra, o, s0);
                    gst<float>(rt, o, s1);
                    gst<float>((void *)row_ptr<float>(D.lo, 0, D.plane, nz, 2, k), o, e0);
                    gst<float>((void *)row_ptr<float>(D.lo, 1, D.plane, nz, 2, k), o, e1);
                } else {
                    gst<float>(ra, o, (float)((AR)ba + ia.p[0]));
                    gst<float>(rt, o, (float)((AR)bt + it.p[0]));
                }
            } else {
                gst<double>(ra, o, (double)((AR)ba + ia.p[0]));
                gst<double>(rt, o, (double)((AR)bt + it.p[0]));
            }
        }
#pragma unroll
        for (int t = 0; t < W - 1; ++t) Wa[t] = Wa[t + 1];
    };
    march_rows<In, prefetch_of<V, AR, ND, COMP>(), FDETD_ROW_UNROLL * prefetch_of<V, AR, ND, COMP>()>(k0, k1, fetch, row, fill);
}

template <typename V, int ND, bool COMP, bool INC, bool AXIS>
__device__ __forceinline__ void envelope_tile(const BatchArgs &A, int t, typename elem<V>::E *lds)
{
    constexpr int S = elem<V>::S, CPW = WAVE / S;
    const int p = problem_of_tile<AXIS>(A, t);
    CDesc &D = ((CDesc *)A.probs)[p];
    TileCoord tc;
    if (!decode_tile(D, t - (AXIS ? D.tile_begin_ax : D.tile_begin), 1, AXIS, CPW, tc)) return;
    const int i0 = tc.i0, k0 = tc.k0, k1 = tc.k1;
    EnvCtx C;
    C.D = &D;
    const bool first = A.n == A.N - 1;
    const size_t pb = D.plane * sizeof(typename stor<V>::T);
    C.psi_a = A.psi[p];
    C.psi_t = A.aux[p];
    const void *ib = D.buf[(A.N - 2 - A.n) & 1], *ob = D.buf[(A.N - 1 - A.n) & 1];
    C.hi_a = C.psi_a;
    C.hi_t = C.psi_t;
    if constexpr (INC) {
        // increment form (no source: d_N = 0): the psi slots hold P = H_a psi.  Role 1: P = H_a lo (from
        // the zero planes); role 2: P += H_a psi_hi in place; stages read d_{n+1}, the first the zero
        // planes; the last adds d_0 into (psi_hi, lo) in place.
        const char *pbuf = (const char *)D.pbuf, *zero = (const char *)D.zero;
        const char *lo = (const char *)D.lo;
        if (A.role == 1) {
            C.vin_a = lo;
            C.vin_t = lo + pb;
            C.psi_a = zero;
            C.psi_t = zero + pb;
            C.out_a = (void *)pbuf;
            C.out_t = (void *)(pbuf + pb);
        } else if (A.role == 2) {
            C.vin_a = C.hi_a;
            C.vin_t = C.hi_t;
            C.psi_a = pbuf;
            C.psi_t = pbuf + pb;
            C.out_a = (void *)pbuf;
            C.out_t = (void *)(pbuf + pb);
        } else {
            C.vin_a = first ? (const void *)zero : ib;
            C.vin_t = first ? (const void *)(zero + pb) : (const char *)ib + pb;
            C.psi_a = pbuf;
            C.psi_t = pbuf + pb;
            C.out_a = A.n == 0 ? (void *)C.hi_a : (void *)ob;
            C.out_t = A.n == 0 ? (void *)C.hi_t : (void *)((const char *)ob + pb);
        }
    } else {
        C.vin_a = first ? C.psi_a : ib;
        C.vin_t = first ? C.psi_t : (const char *)ib + pb;
        const bool in_place = A.n == 0 && A.N > 1;
        C.out_a = in_place ? (void *)C.psi_a : (void *)ob;
        C.out_t = in_place ? (void *)C.psi_t : (void *)((const char *)ob + pb);
    }
    C.chi = A.chi[p];
    C.compensated = A.compensated && A.n == 0 && A.role == 0;
    C.coef = A.coef;
    using AR = typename std::conditional<AXIS, double, typename scal<V>::R>::type;
    env_march<V, AR, ND, COMP, INC>(C, i0, k0, k1, lds);
}

template <typename V, int ND, bool COMP, bool INC>
__global__ __launch_bounds__(WAVE) void k_envelope_stage(BatchArgs A)
{
    using VA = typename std::conditional<(ND <= kAxisWholeND), float2, f2pair>::type;
    __shared__ __align__(16) unsigned char smem[cmax(lds_row_bytes<V, ND>(), lds_row_bytes<VA, ND>())];
    bool axis;
    const int t = tile_of_block(A.ntiles_ax, A.ntiles, axis);
    if (t < 0) return;
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if (axis) {
            envelope_tile<VA, ND, COMP, INC, true>(A, t, (typename elem<VA>::E *)smem);
            return;
        }
    }
    envelope_tile<V, ND, COMP, INC, false>(A, t, (typename elem<V>::E *)smem);
}

// --------------------------------------------------------------------------------------------------
// Current staging (section 2.5): Jbar_rho = S_rho^(-) J_rho on the rho-staggered rows k >= 1 (row 0 = 0),
// the half-shift with the m_A mirror ghosts of section 2.4, in FP64 arithmetic.  J_theta and J_z are read
// by the stages as they are.  Same tiling as the stage launch of the batch; only the tiles of the first
// half carry work.  Window: primary rows q = k - N_D .. k + N_D - 1 of J_rho.
// --------------------------------------------------------------------------------------------------
template <typename V>
__device__ __forceinline__ void store_value(void *row, unsigned o, const lv<double, elem<V>::K> &x)
{
    if constexpr (std::is_same<typename elem<V>::E, float2>::value) gst<float2>(row, o, float2{(float)x.p[0], (float)x.p[1]});
    else if constexpr (std::is_same<typename elem<V>::E, float>::value) gst<float>(row, o, (float)x.p[0]);
    else gst<double>(row, o, x.p[0]);
}

template <typename V, int ND, bool AXIS>
__device__ __forceinline__ void stagger_tile(const BatchArgs &A, int t)
{
    constexpr int S = elem<V>::S, K = elem<V>::K, CPW = WAVE / S;
    using E = typename elem<V>::E;
    using SV = typename stor<V>::T;
    using L_ = lv<double, K>;
    const int p = problem_of_tile<AXIS>(A, t);
    CDesc &D = ((CDesc *)A.probs)[p];
    TileCoord tc;
    if (!decode_tile(D, t - (AXIS ? D.tile_begin_ax : D.tile_begin), 2, AXIS, CPW, tc) || tc.half) return;
    const int k0 = tc.k0, k1 = tc.k1, nz = D.nz, nr = D.nr;
    const Lane<V> L(tc.i0, nz);
    const SV *jr = (const SV *)A.aux[p];
    const double pA = -D.pS;
    const L_ zero = zero_lv<double, K>();
    L_ W[2 * ND];
    auto fill = [&]() {
#pragma unroll
        for (int t2 = 0; t2 < 2 * ND - 1; ++t2) {
            const int q = k0 - ND + t2;
            W[t2] = ldrow<V, double>(jr, nz, min(q < 0 ? -1 - q : q, nr - 1), L);
        }
#pragma unroll
        for (int t2 = 0; t2 < 2 * ND - 1; ++t2) {
            const int q = k0 - ND + t2;
            W[t2] = q >= nr ? zero : (q < 0 ? pA : 1.0) * W[t2];
        }
    };
    struct In {
        E j;
    };
    auto fetch = [&](int k) -> In {
        const int qn = k + ND - 1;
        return In{ldraw<V>(jr, nz, qn < nr ? qn : nr - 1, L)};
    };
    auto row = [&](const In &cu, int k, bool live) {
        const int qn = k + ND - 1;
        W[2 * ND - 1] = keep_if(qn < nr, to_lv<double>(cu.j));
        L_ s = zero;
#pragma unroll
        for (int j = 1; j <= ND; ++j) s = fmav((double)D.sh[j - 1], W[ND + j - 1] + W[ND - j], s);
        if (L.col && live)
            store_value<V>((void *)row_ptr<E>(D.jbar, 0, 0, nz, S, k), (unsigned)L.eidx, k == 0 ? zero : s);
#pragma unroll
        for (int t2 = 0; t2 < 2 * ND - 1; ++t2) W[t2] = W[t2 + 1];
    };
    march_rows<In, FDETD_PREFETCH, FDETD_PREFETCH>(k0, k1, fetch, row, fill);
}

template <typename V, int ND>
__global__ __launch_bounds__(WAVE) void k_stagger_march(BatchArgs A)
{
    bool axis;
    const int t = tile_of_block(A.ntiles_ax, A.ntiles, axis);
    if (t < 0) return;
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if (axis) {
            stagger_tile<typename std::conditional<(ND <= kAxisWholeND), float2, f2pair>::type, ND, true>(A, t);
            return;
        }
    }
    stagger_tile<V, ND, false>(A, t);
}

template <typename V, int ND>
hipError_t go_stagger(const BatchArgs &a, hipStream_t s)
{
    if (sizeof(typename scal<V>::R) == 8 && a.ntiles_ax) return hipErrorInvalidValue;  // FP32 storage only
    hipLaunchKernelGGL((k_stagger_march<V, ND>), dim3(blocks_of(a.ntiles_ax, a.ntiles)), dim3(WAVE), 0, s, a);
    return hipGetLastError();
}

// Launch stage n of a batch with the kernel variant its flags select.
// The Horner form (INC false) also exists with non-temporal output stores (the plan's choice per batch).
template <typename V, int ND, bool SRC, bool COMP, bool INC, bool WN = false>
hipError_t go_maxwell_v(const BatchArgs &a, hipStream_t s)
{
    if (sizeof(typename scal<V>::R) == 8 && a.ntiles_ax) return hipErrorInvalidValue;  // FP32 storage only
    const dim3 grid(blocks_of(a.ntiles_ax, a.ntiles));
    if constexpr (!INC) {
        if (a.nt_store) {
            hipLaunchKernelGGL((k_maxwell_stage<V, ND, SRC, COMP, false, WN, true>), grid, dim3(WAVE), 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL((k_maxwell_stage<V, ND, SRC, COMP, INC, WN, false>), grid, dim3(WAVE), 0, s, a);
    return hipGetLastError();
}

template <typename V, int ND, bool INC>
hipError_t go_maxwell_i(const BatchArgs &a, hipStream_t s)
{
    const bool comp = sizeof(typename scal<V>::R) == 4 && a.compensated && a.n == 0 && a.role == 0;
    if (comp) {
        if constexpr (sizeof(typename scal<V>::R) == 4) {
            if (a.has_src) return go_maxwell_v<V, ND, true, true, INC>(a, s);
            return go_maxwell_v<V, ND, false, true, INC>(a, s);
        }
    }
    if (a.has_src) {
        // the first stage of a step with a current forms w_N itself when the plan left out the w_N pass
        if constexpr (!INC)
            if (a.fuse_wn && a.n == a.N - 1) return go_maxwell_v<V, ND, true, false, false, true>(a, s);
        return go_maxwell_v<V, ND, true, false, INC>(a, s);
    }
    return go_maxwell_v<V, ND, false, false, INC>(a, s);
}

// The increment form exists for FP32 storage (FP32C plans) only.
template <typename V, int ND>
hipError_t go_maxwell(const BatchArgs &a, hipStream_t s)
{
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if (a.increment) return go_maxwell_i<V, ND, true>(a, s);
    } else {
        if (a.increment) return hipErrorInvalidValue;
    }
    return go_maxwell_i<V, ND, false>(a, s);
}

template <typename V, int ND, bool COMP, bool INC>
hipError_t go_envelope_v(const BatchArgs &a, hipStream_t s)
{
    if (sizeof(typename scal<V>::R) == 8 && a.ntiles_ax) return hipErrorInvalidValue;  // FP32 storage only
    hipLaunchKernelGGL((k_envelope_stage<V, ND, COMP, INC>), dim3(blocks_of(a.ntiles_ax, a.ntiles)), dim3(WAVE), 0,
                       s, a);
    return hipGetLastError();
}

// The increment form exists for FP32 storage (FP32C plans) only.
template <typename V, int ND>
hipError_t go_envelope(const BatchArgs &a, hipStream_t s)
{
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        const bool comp = a.compensated && a.n == 0 && a.role == 0;
        if (a.increment) return comp ? go_envelope_v<V, ND, true, true>(a, s) : go_envelope_v<V, ND, false, true>(a, s);
        if (comp) return go_envelope_v<V, ND, true, false>(a, s);
    } else {
        if (a.increment) return hipErrorInvalidValue;
    }
    return go_envelope_v<V, ND, false, false>(a, s);
}

// --------------------------------------------------------------------------------------------------
// Launches that mix stencil widths: every problem of the batch keeps its own N_D, and each tile runs the
// code specialised for its problem's N_D (the same code, and so the same results, as the per-width
// launches).  One launch per stage for all problems of equal Taylor order and time step.
// --------------------------------------------------------------------------------------------------
#ifdef FDETD_ANY_WIDTH
template <typename V, bool SRC, bool COMP, bool AXIS, bool WN, int ND>
__device__ __forceinline__ void stage_tile_any(const BatchArgs &A, int t, unsigned char *smem)
{
    using VA = typename std::conditional<(ND <= kAxisWholeND), float2, f2pair>::type;
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if constexpr (AXIS) {
            using EA = typename elem<VA>::E;
            maxwell_tile<VA, ND, SRC, COMP, false, true, WN, false>(A, t, (EA(*)[WAVE + 2 * ND * elem<VA>::S])smem);
            return;
        }
    }
    using E = typename elem<V>::E;
    maxwell_tile<V, ND, SRC, COMP, false, false, WN, false>(A, t, (E(*)[WAVE + 2 * ND * elem<V>::S])smem);
}

// AXIS: the launch covers the FP32C near-axis tiles only (their FP64-arithmetic code for all widths in one
// kernel would not fit the registers of two wavefronts per SIMD); otherwise the main tiles only.
template <typename V, bool SRC, bool COMP, bool AXIS, bool WN>
__global__ __launch_bounds__(WAVE) void k_maxwell_stage_any(BatchArgs A)
{
    __shared__ __align__(16) unsigned char smem[cmax(stage_lds_bytes<V, kMaxND>(), stage_lds_bytes<f2pair, kMaxND>())];
    bool axis;
    const int t = tile_of_block(A.ntiles_ax, A.ntiles, axis);
    if (t < 0 || axis != AXIS) return;
    const int p = problem_of_tile<AXIS>(A, t);
    switch (((CDesc *)A.probs)[p].nd) {
#define FDETD_C(N) \
    case N: stage_tile_any<V, SRC, COMP, AXIS, WN, N>(A, t, smem); break;
        FDETD_C(1) FDETD_C(2) FDETD_C(3) FDETD_C(4) FDETD_C(5) FDETD_C(6) FDETD_C(7) FDETD_C(8) FDETD_C(9) FDETD_C(10)
        FDETD_C(11) FDETD_C(12) FDETD_C(13) FDETD_C(14) FDETD_C(15) FDETD_C(16)
#undef FDETD_C
    default: break;
    }
}

template <typename V>
__global__ __launch_bounds__(WAVE) void k_stagger_march_any(BatchArgs A)
{
    bool axis;
    const int t = tile_of_block(A.ntiles_ax, A.ntiles, axis);
    if (t < 0) return;
    const int p = axis ? problem_of_tile<true>(A, t) : problem_of_tile<false>(A, t);
    switch (((CDesc *)A.probs)[p].nd) {
#define FDETD_C(N)                                                                                                    \
    case N:                                                                                                           \
        if constexpr (sizeof(typename scal<V>::R) == 4) {                                                              \
            if (axis) {                                                                                                \
                stagger_tile<typename std::conditional<(N <= kAxisWholeND), float2, f2pair>::type, N, true>(A, t);   \
                break;                                                                                                 \
            }                                                                                                          \
        }                                                                                                              \
        stagger_tile<V, N, false>(A, t);                                                                               \
        break;
        FDETD_C(1) FDETD_C(2) FDETD_C(3) FDETD_C(4) FDETD_C(5) FDETD_C(6) FDETD_C(7) FDETD_C(8) FDETD_C(9) FDETD_C(10)
        FDETD_C(11) FDETD_C(12) FDETD_C(13) FDETD_C(14) FDETD_C(15) FDETD_C(16)
#undef FDETD_C
    default: break;
    }
}

// The main tiles, then (FP32 storage) the near-axis tiles in a second launch.
template <typename V, bool SRC, bool COMP, bool WN = false>
hipError_t go_maxwell_any_v(const BatchArgs &a, hipStream_t s)
{
    if (sizeof(typename scal<V>::R) == 8 && a.ntiles_ax) return hipErrorInvalidValue;  // FP32 storage only
    BatchArgs m = a;
    m.ntiles_ax = 0;
    if (m.ntiles) hipLaunchKernelGGL((k_maxwell_stage_any<V, SRC, COMP, false, WN>), dim3(blocks_of(0, m.ntiles)), dim3(WAVE), 0, s, m);
    if constexpr (sizeof(typename scal<V>::R) == 4) {
        if (a.ntiles_ax) {
            BatchArgs x = a;
            x.ntiles = 0;
            hipLaunchKernelGGL((k_maxwell_stage_any<V, SRC, COMP, true, WN>), dim3(blocks_of(x.ntiles_ax, 0)), dim3(WAVE), 0, s, x);
        }
    }
    return hipGetLastError();
}
#endif

}  // namespace

// Per-N_D entry points; fdetd_march.hip is compiled once per N_D range (FDETD_ND_LO .. FDETD_ND_HI) so
// that the many kernel variants build in parallel.
#define FDETD_MARCH_INST(N)                                                                          \
    template <>                                                                                      \
    hipError_t march_maxwell_nd<N>(int prec, const BatchArgs &a, hipStream_t s)                      \
    {                                                                                                \
        return prec == P64 ? go_maxwell<double2, N>(a, s) : go_maxwell<float2, N>(a, s);             \
    }                                                                                                \
    template <>                                                                                      \
    hipError_t march_envelope_nd<N>(int prec, const BatchArgs &a, hipStream_t s)                     \
    {                                                                                                \
        return prec == P64 ? go_envelope<double2, N>(a, s) : go_envelope<float2, N>(a, s);           \
    }                                                                                                \
    template <>                                                                                      \
    hipError_t march_stagger_nd<N>(int prec, const BatchArgs &a, hipStream_t s)                      \
    {                                                                                                \
        return prec == P64 ? go_stagger<double2, N>(a, s) : go_stagger<float2, N>(a, s);             \
    }

#ifndef FDETD_ND_LO
#define FDETD_ND_LO 1
#define FDETD_ND_HI 16
#endif
#ifdef FDETD_ANY_WIDTH
// FDETD_ANY_WIDTH = 0: FP64 launches; 1: FP32 storage without, 2: with the compensated last stage
#if FDETD_ANY_WIDTH == 0
hipError_t march_maxwell_any_p64(const BatchArgs &a, hipStream_t s)
{
    if (!a.has_src) return go_maxwell_any_v<double2, false, false>(a, s);
    return a.fuse_wn && a.n == a.N - 1 ? go_maxwell_any_v<double2, true, false, true>(a, s)
                                       : go_maxwell_any_v<double2, true, false>(a, s);
}
hipError_t march_stagger_any_p64(const BatchArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_stagger_march_any<double2>, dim3(blocks_of(a.ntiles_ax, a.ntiles)), dim3(WAVE), 0, s, a);
    return hipGetLastError();
}
#elif FDETD_ANY_WIDTH == 1
hipError_t march_maxwell_any_p32(const BatchArgs &a, hipStream_t s)
{
    if (!a.has_src) return go_maxwell_any_v<float2, false, false>(a, s);
    return a.fuse_wn && a.n == a.N - 1 ? go_maxwell_any_v<float2, true, false, true>(a, s)
                                       : go_maxwell_any_v<float2, true, false>(a, s);
}
hipError_t march_stagger_any_p32(const BatchArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_stagger_march_any<float2>, dim3(blocks_of(a.ntiles_ax, a.ntiles)), dim3(WAVE), 0, s, a);
    return hipGetLastError();
}
#else
hipError_t march_maxwell_any_p32c(const BatchArgs &a, hipStream_t s)
{
    return a.has_src ? go_maxwell_any_v<float2, true, true>(a, s) : go_maxwell_any_v<float2, false, true>(a, s);
}
#endif
#endif
#if FDETD_ND_LO <= 1 && 1 <= FDETD_ND_HI
FDETD_MARCH_INST(1)
#endif
#if FDETD_ND_LO <= 2 && 2 <= FDETD_ND_HI
FDETD_MARCH_INST(2)
#endif
#if FDETD_ND_LO <= 3 && 3 <= FDETD_ND_HI
FDETD_MARCH_INST(3)
#endif
#if FDETD_ND_LO <= 4 && 4 <= FDETD_ND_HI
FDETD_MARCH_INST(4)
#endif
#if FDETD_ND_LO <= 5 && 5 <= FDETD_ND_HI
FDETD_MARCH_INST(5)
#endif
#if FDETD_ND_LO <= 6 && 6 <= FDETD_ND_HI
FDETD_MARCH_INST(6)
#endif
#if FDETD_ND_LO <= 7 && 7 <= FDETD_ND_HI
FDETD_MARCH_INST(7)
#endif
#if FDETD_ND_LO <= 8 && 8 <= FDETD_ND_HI
FDETD_MARCH_INST(8)
#endif
#if FDETD_ND_LO <= 9 && 9 <= FDETD_ND_HI
FDETD_MARCH_INST(9)
#endif
#if FDETD_ND_LO <= 10 && 10 <= FDETD_ND_HI
FDETD_MARCH_INST(10)
#endif
#if FDETD_ND_LO <= 11 && 11 <= FDETD_ND_HI
FDETD_MARCH_INST(11)
#endif
#if FDETD_ND_LO <= 12 && 12 <= FDETD_ND_HI
FDETD_MARCH_INST(12)
#endif
#if FDETD_ND_LO <= 13 && 13 <= FDETD_ND_HI
FDETD_MARCH_INST(13)
#endif
#if FDETD_ND_LO <= 14 && 14 <= FDETD_ND_HI
FDETD_MARCH_INST(14)
#endif
#if FDETD_ND_LO <= 15 && 15 <= FDETD_ND_HI
FDETD_MARCH_INST(15)
#endif
#if FDETD_ND_LO <= 16 && 16 <= FDETD_ND_HI
FDETD_MARCH_INST(16)
#endif

}  // namespace fdetd
