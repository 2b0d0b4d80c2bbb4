// fdetd_step_noalloc: the Maxwell step of one problem without a plan and without any device allocation,
// for callers that cannot allocate (code under graph capture, serving loops).  Everything a plan would own
// -- the problem descriptor, the 1/rho tables, the two stage vectors, the staged current and the FP32C
// compensation words -- lives in one static device array of fixed size, `scratch`.  Each device the
// library runs on holds its own copy of the array at its own address, obtained once per device with
// hipGetSymbolAddress; host code uses only that address, never the array's name.
//
// The step is the one fdetd_step enqueues (section 2.1 midpoint solution in the Horner form of the
// algorithm summary of section 2.5, current staged with S_rho^(-,mA), axis rule of section 2.4), on the
// same kernels, so the results are the same bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "../../include/fdetd.h"
#include "fdetd_internal.h"

namespace fdetd {
namespace {

constexpr size_t kNoAllocMaxCells = size_t(1) << 16;  // nz * nr
constexpr int kNoAllocMaxRows = 4096;                  // nr
constexpr size_t kAlign = 256;
constexpr size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
// descriptor, two 1/rho tables, two 6-plane stage vectors, the staged J_rho plane (all at 16 B per complex
// value in FP64) and the FP32C compensation words (6 planes of float2, fewer bytes than FP64 planes save)
constexpr size_t kScratchBytes = align_up(sizeof(ProbDesc)) + 2 * align_up(kNoAllocMaxRows * sizeof(double)) +
                                 2 * align_up(6 * kNoAllocMaxCells * 16) + align_up(kNoAllocMaxCells * 16);

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void *g_ptr[kMaxDevices];  // device address of scratch on each device (null until set up)

// the message goes where fdetd_last_error(NULL) reads it
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    set_last_error(buf);
    return code;
}

// The device address of scratch on the current device, looked up on the first call on that device.
int scratch_of_device(void **out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(FDETD_E_HIP, "fdetd_step_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(FDETD_E_ARG, "fdetd_step_noalloc: device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(FDETD_E_HIP, "fdetd_step_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return FDETD_OK;
}

// Writes the descriptor (passed by value, no host-to-device copy), the 1/rho tables, and zeroes the FP32C
// compensation words (a kernel, not a memset, so that the call can be captured into a graph).
__global__ __launch_bounds__(256) void k_noalloc_setup(ProbDesc D, ProbDesc *dst, double *rinv_p, double *rinv_s,
                                                       float *lo, size_t nlo)
{
    const size_t t = (size_t)blockIdx.x * 256 + threadIdx.x, stride = (size_t)gridDim.x * 256;
    static_assert(sizeof(ProbDesc) % 8 == 0, "descriptor copied in 8-byte words");
    const unsigned long long *src = (const unsigned long long *)&D;
    for (size_t w = t; w < sizeof(ProbDesc) / 8; w += stride) ((unsigned long long *)dst)[w] = src[w];
    for (size_t k = t; k < (size_t)D.nr; k += stride) {
        rinv_p[k] = 1.0 / ((k + 0.5) * D.dr);
        rinv_s[k] = k ? 1.0 / (k * D.dr) : 0.0;
    }
    for (size_t q = t; lo && q < nlo; q += stride) lo[q] = 0.f;
}

}  // namespace
}  // namespace fdetd

using namespace fdetd;

extern "C" FDETD_API int fdetd_step_noalloc(const fdetd_problem_desc *prob, int32_t precision, void *stream, void *psi,
                                            const void *j_half, int64_t j_step_blocks, int32_t n_steps)
{
    if (!prob) return fail(FDETD_E_ARG, "fdetd_step_noalloc: prob is NULL");
    const fdetd_problem_desc &d = *prob;
    const int nd = d.fd_order / 2;
    if (d.kind != FDETD_MAXWELL) return fail(FDETD_E_ARG, "fdetd_step_noalloc: not a Maxwell problem");
    if (precision != FDETD_FP64 && precision != FDETD_FP32C)
        return fail(FDETD_E_ARG, "fdetd_step_noalloc: unknown precision %d", precision);
    if (d.fd_order < 2 || d.fd_order > 2 * kMaxND || (d.fd_order & 1) || d.nz < 2 * nd + 1 || d.nr < nd + 1 ||
        d.m < 0 || d.m > 64 || d.taylor_order < 1 || d.taylor_order > 32 || !(d.dz > 0) || !(d.dr > 0) ||
        !(d.dt > 0) || !std::isfinite(d.dz + d.dr + d.dt))
        return fail(FDETD_E_ARG, "fdetd_step_noalloc: bad problem (sizes, orders, mode or steps)");
    const size_t cells = (size_t)d.nz * d.nr;
    if (cells > kNoAllocMaxCells || d.nr > kNoAllocMaxRows)
        return fail(FDETD_E_ARG, "fdetd_step_noalloc: grid %d x %d exceeds the scratch limit of %zu cells and %d rows",
                    d.nz, d.nr, kNoAllocMaxCells, kNoAllocMaxRows);
    const size_t eb = precision == FDETD_FP64 ? 16 : 8;
    if (!psi || (uintptr_t)psi % eb || (j_half && (uintptr_t)j_half % eb) || n_steps < 0 || j_step_blocks < 0)
        return fail(FDETD_E_ARG, "fdetd_step_noalloc: NULL or misaligned pointer, or negative counts");
    if (n_steps == 0) return FDETD_OK;
    void *base = nullptr;
    int rc = scratch_of_device(&base);
    if (rc) return rc;

    // scratch layout (each part 256-byte aligned)
    char *p = (char *)base;
    ProbDesc *ddesc = (ProbDesc *)p;
    p += align_up(sizeof(ProbDesc));
    double *rinv_p = (double *)p;
    p += align_up(kNoAllocMaxRows * sizeof(double));
    double *rinv_s = (double *)p;
    p += align_up(kNoAllocMaxRows * sizeof(double));
    void *buf0 = p;
    p += align_up(6 * cells * eb);
    void *buf1 = p;
    p += align_up(6 * cells * eb);
    void *jbar = p;
    p += align_up(cells * eb);
    float *lo = precision == FDETD_FP32C ? (float *)p : nullptr;
    p += precision == FDETD_FP32C ? align_up(6 * cells * 8) : 0;
    if ((size_t)(p - (char *)base) > kScratchBytes) return fail(FDETD_E_ARG, "fdetd_step_noalloc: internal: scratch layout");

    ProbDesc D;
    describe_problem(d, precision, default_segment_rows(precision, d), D);
    D.buf[0] = buf0;
    D.buf[1] = buf1;
    D.jbar = jbar;
    D.lo = lo;
    D.rinv_p = rinv_p;
    D.rinv_s = rinv_s;
    const hipStream_t s = (hipStream_t)stream;
    const int prec = precision == FDETD_FP64 ? P64 : P32;
    hipLaunchKernelGGL(k_noalloc_setup, dim3(64), dim3(256), 0, s, D, ddesc, rinv_p, rinv_s, lo, 2 * 6 * cells);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(FDETD_E_HIP, "fdetd_step_noalloc: setup: %s", hipGetErrorString(e));

    BatchArgs A;
    std::memset(&A, 0, sizeof A);
    A.probs = ddesc;
    A.nprob = 1;
    A.ntiles = 2 * D.nseg * D.nstrip;
    A.ntiles_ax = 2 * D.nseg_ax * D.nstrip_ax;
    A.N = d.taylor_order;
    A.has_src = j_half != nullptr;
    A.compensated = precision == FDETD_FP32C;
    A.psi[0] = psi;
    const int N = d.taylor_order;
    // the first stage forms w_N as it loads psi and Jbar, except FP32C at N = 1 (its first stage is the
    // compensated last one): then a pass of its own writes w_N first
    A.fuse_wn = j_half != nullptr && !(precision == FDETD_FP32C && N == 1);
    for (int st = 0; st < n_steps; ++st) {
        A.aux[0] = j_half ? (const char *)j_half + (size_t)(j_step_blocks * st) * 3 * cells * eb : nullptr;
        A.beta_in = -d.dt * std::ldexp(1.0, -N);
        if (j_half) {
            if ((e = launch_stagger_march(prec, nd, A, s)) != hipSuccess ||
                (!A.fuse_wn && (e = launch_form_wn(prec, A, cells, s)) != hipSuccess))
                return fail(FDETD_E_HIP, "fdetd_step_noalloc: current staging: %s", hipGetErrorString(e));
        }
        for (int n = N - 1; n >= 0; --n) {
            A.n = n;
            A.beta = -d.dt * std::ldexp(1.0, -n);
            A.coef = d.dt / (n + 1);
            if ((e = launch_maxwell_march(prec, nd, A, s)) != hipSuccess)
                return fail(FDETD_E_HIP, "fdetd_step_noalloc: stage: %s", hipGetErrorString(e));
        }
        if (N == 1 && (e = launch_copy(buf0, psi, 6 * cells * eb, s)) != hipSuccess)
            return fail(FDETD_E_HIP, "fdetd_step_noalloc: copy: %s", hipGetErrorString(e));
    }
    AxisArgs X{};
    X.psi = psi;
    X.nz = d.nz;
    X.nr = d.nr;
    X.m = d.m;
    for (int u = 0; u < nd; ++u) X.cax[u] = D.cax[u];
    if ((e = launch_axis_fix(prec, nd, X, s)) != hipSuccess)
        return fail(FDETD_E_HIP, "fdetd_step_noalloc: axis rule: %s", hipGetErrorString(e));
    return FDETD_OK;
}

