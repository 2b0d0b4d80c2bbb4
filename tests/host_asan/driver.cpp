// Host-only driver of the library's C-ABI for a sanitizer build: every call here returns before any HIP
// call (argument checks, coefficient tables, the stability bound), so it runs without a GPU.  The kernels
// are replaced by stubs that are never reached.
#include <cmath>
#include <cstdio>
#include <cstring>

#include "fdetd.h"
#include "fdetd_internal.h"

namespace fdetd {
#define STUB_ND(N)                                                                                        \
    template <> hipError_t march_maxwell_nd<N>(int, const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; } \
    template <> hipError_t march_envelope_nd<N>(int, const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; } \
    template <> hipError_t march_stagger_nd<N>(int, const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
STUB_ND(1) STUB_ND(2) STUB_ND(3) STUB_ND(4) STUB_ND(5) STUB_ND(6) STUB_ND(7) STUB_ND(8)
STUB_ND(9) STUB_ND(10) STUB_ND(11) STUB_ND(12) STUB_ND(13) STUB_ND(14) STUB_ND(15) STUB_ND(16)
#undef STUB_ND
hipError_t launch_maxwell_stage(int, int, const MaxwellStageArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_envelope_stage(int, int, const EnvelopeStageArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_axis_fix(int, int, const AxisArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_deposit_jz(int, const DepositArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_deposit_rho(int, const DepositArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_deposit_current(int, const DepositArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_absorb_damp(int, const DampArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_destagger(int, const DestaggerArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_envelope_gather(int, const EnvGatherArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_ponderomotive(int, const ProbDesc *, int, int, int, const void *, void *, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_correct_div(int, const CorrectArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_correct_apply(int, const CorrectArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_correct_solve(const SolveArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_gather(int, const GatherArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_gather_box(const double *, int64_t, int, int, double, double, int *, int *, int, hipStream_t)
{
    return hipErrorInvalidValue;
}
hipError_t launch_norm2(int, const void *, size_t, double *, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_scale(int, void *, size_t, double, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_copy(const void *, void *, size_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_form_wn(int, const BatchArgs &, size_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_jgen(int, const JgenArgs &, size_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_axis_fix_batch(int, const BatchArgs &, int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t march_maxwell_any_p64(const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t march_maxwell_any_p32(const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t march_maxwell_any_p32c(const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t march_stagger_any_p64(const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
hipError_t march_stagger_any_p32(const BatchArgs &, hipStream_t) { return hipErrorInvalidValue; }
}  // namespace fdetd

static int failures = 0;
#define EXPECT(c)                                                              \
    do {                                                                       \
        if (!(c)) {                                                            \
            std::printf("FAILED %s:%d: %s\n", __FILE__, __LINE__, #c);         \
            ++failures;                                                        \
        }                                                                      \
    } while (0)

static fdetd_problem_desc good()
{
    fdetd_problem_desc d;
    std::memset(&d, 0, sizeof d);
    d.kind = FDETD_MAXWELL;
    d.nz = 64;
    d.nr = 16;
    d.m = 1;
    d.fd_order = 8;
    d.taylor_order = 8;
    d.dz = 0.3;
    d.dr = 0.6;
    d.dt = 0.15;
    d.k0 = 1.0;
    return d;
}

int main()
{
    // coefficient tables: every table and width, and the rejected ones
    double out[17];
    for (int which = 0; which <= 4; ++which)
        for (int nd = 1; nd <= 16; ++nd) {
            EXPECT(fdetd_coefficients(which, nd, out) == FDETD_OK);
            for (int j = 0; j < nd; ++j) EXPECT(std::isfinite(out[j]));
        }
    EXPECT(fdetd_coefficients(5, 4, out) == FDETD_E_ARG);
    EXPECT(fdetd_coefficients(0, 0, out) == FDETD_E_ARG);
    EXPECT(fdetd_coefficients(0, 17, out) == FDETD_E_ARG);
    EXPECT(fdetd_coefficients(0, 4, nullptr) == FDETD_E_ARG);
    for (int N = 1; N <= 32; ++N) EXPECT(fdetd_taylor_stability_bound(N) >= 0.0);
    // plan arguments rejected before any device work
    fdetd_plan_t P = nullptr;
    fdetd_problem_desc d = good();
    EXPECT(fdetd_plan(&d, 1, FDETD_FP64, 0, nullptr, nullptr) == FDETD_E_ARG);
    EXPECT(fdetd_plan(nullptr, 1, FDETD_FP64, 0, nullptr, &P) == FDETD_E_ARG && !P);
    EXPECT(fdetd_plan(&d, 0, FDETD_FP64, 0, nullptr, &P) == FDETD_E_ARG && !P);
    EXPECT(fdetd_plan(&d, 1, 7, 0, nullptr, &P) == FDETD_E_ARG && !P);
    EXPECT(fdetd_plan(&d, 1, FDETD_FP64, FDETD_PLAN_USE_GRAPH, nullptr, &P) == FDETD_E_ARG && !P);
    const char *msg = fdetd_last_error(nullptr);
    EXPECT(msg && std::strlen(msg) > 0);
    fdetd_problem_desc bad[12];
    for (auto &b : bad) b = good();
    bad[0].nz = 8;           // < 2 N_D + 1
    bad[1].nr = 4;           // < N_D + 1
    bad[2].fd_order = 7;     // odd
    bad[3].fd_order = 34;    // > 32
    bad[4].m = -1;
    bad[5].m = 65;
    bad[6].taylor_order = 0;
    bad[7].taylor_order = 33;
    bad[8].dt = 0.0;
    bad[9].dz = -1.0;
    bad[10].dr = NAN;
    bad[11].kind = 5;
    for (auto &b : bad) EXPECT(fdetd_plan(&b, 1, FDETD_FP64, 0, nullptr, &P) == FDETD_E_ARG && !P);
    fdetd_problem_desc mixed[2] = {good(), good()};
    mixed[1].kind = FDETD_ENVELOPE;
    EXPECT(fdetd_plan(mixed, 2, FDETD_FP64, 0, nullptr, &P) == FDETD_E_ARG && !P);
    fdetd_problem_desc env = good();
    env.kind = FDETD_ENVELOPE;
    EXPECT(fdetd_plan(&env, 1, FDETD_FP64, FDETD_PLAN_CURRENT_CORRECTION, nullptr, &P) == FDETD_E_ARG && !P);
    // calls on a NULL plan
    void *ptrs[1] = {nullptr};
    EXPECT(fdetd_step(nullptr, ptrs, nullptr, 0, 1) == FDETD_E_ARG);
    EXPECT(envelope_step(nullptr, ptrs, ptrs, ptrs, 0, 1) == FDETD_E_ARG);
    EXPECT(fdetd_deposit_jz(nullptr, nullptr, 0, 1.0, 0.5, ptrs) == FDETD_E_ARG);
    EXPECT(fdetd_deposit_rho(nullptr, nullptr, 0, 0.0, 0.5, ptrs) == FDETD_E_ARG);
    EXPECT(fdetd_deposit_current(nullptr, nullptr, 0, 0.5, ptrs) == FDETD_E_ARG);
    EXPECT(envelope_absorber(nullptr, -1, 4, 4, 1.0, 2.0) == FDETD_E_ARG);
    EXPECT(fdetd_gather(nullptr, ptrs, nullptr, 0, nullptr) == FDETD_E_ARG);
    EXPECT(envelope_ponderomotive(nullptr, ptrs, ptrs) == FDETD_E_ARG);
    fdetd_plan_info info;
    EXPECT(fdetd_query(nullptr, &info) == FDETD_E_ARG);
    size_t bytes = 0;
    EXPECT(fdetd_export_state(nullptr, nullptr, &bytes) == FDETD_E_ARG);
    EXPECT(fdetd_import_state(nullptr, nullptr, 0) == FDETD_E_ARG);
    fdetd_destroy(nullptr);
    EXPECT(std::strlen(fdetd_last_error(nullptr)) > 0);
    if (failures == 0) std::printf("host driver ok\n");
    return failures ? 1 : 0;
}
