// C ABI of libqpat: argument checks, context state, allocation, and the
// layout changes between the caller's [n_ill][N] arrays and the interleaved
// [N][n_pad] arrays used inside the library.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <algorithm>

#include <functional>
#include <thread>

#include "qpat_internal.h"

namespace qpat {

qpat_status fail(qpat_ctx* c, qpat_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

qpat_status hip_check(qpat_ctx* c, hipError_t e, const char* what) {
    if (e == hipSuccess) return QPAT_OK;
    return fail(c, e == hipErrorOutOfMemory ? QPAT_ERR_OOM : QPAT_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

qpat_status dfree(qpat_ctx* c, void* p) {
    if (!p) return QPAT_OK;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    QPAT_HIP(c, hipFree(p));
    return QPAT_OK;
}

namespace {

__global__ void k_from_interleaved(int64_t N, int n_ill, int n_pad, const double* __restrict__ src,
                                   const double* __restrict__ mu, double* __restrict__ dst) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * n_ill) return;
    const int64_t k = t / N, row = t % N;
    double v = src[row * n_pad + k];
    if (mu) v *= mu[row];
    dst[t] = v;
}

__global__ void k_copy_d(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) b[i] = a[i];
}

bool pow2_block(int b) { return b == 1 || b == 2 || b == 4 || b == 8 || b == 16; }

qpat_status check_opts(qpat_ctx* c, const qpat_opts* o) {
    if (o->precision != 0 && o->precision != 1) return fail(c, QPAT_ERR_ARG, "precision must be 0 or 1");
    if (!pow2_block(o->max_rhs_block)) return fail(c, QPAT_ERR_ARG, "max_rhs_block must be 1, 2, 4, 8 or 16");
    if (!(o->pcg_rtol > 0.0) || !(o->prior_rtol > 0.0)) return fail(c, QPAT_ERR_ARG, "tolerances must be > 0");
    if (o->pcg_maxit < 1) return fail(c, QPAT_ERR_ARG, "pcg_maxit must be >= 1");
    if (o->lsqr_max_steps < 1) return fail(c, QPAT_ERR_ARG, "lsqr_max_steps must be >= 1");
    if (!(o->ru_delta > 0.0 && o->ru_delta < 1.0)) return fail(c, QPAT_ERR_ARG, "ru_delta must be in (0, 1)");
    if (o->use_graphs != 0 && o->use_graphs != 1) return fail(c, QPAT_ERR_ARG, "use_graphs must be 0 or 1");
    if (o->operator_format != 0 && o->operator_format != 1)
        return fail(c, QPAT_ERR_ARG, "operator_format must be 0 or 1");
    if (o->prior_precond != 0 && o->prior_precond != 1) return fail(c, QPAT_ERR_ARG, "prior_precond must be 0 or 1");
    if (o->pcg_precond != 0 && o->pcg_precond != 1) return fail(c, QPAT_ERR_ARG, "pcg_precond must be 0 or 1");
    if (o->autotune != 0 && o->autotune != 1) return fail(c, QPAT_ERR_ARG, "autotune must be 0 or 1");
    return QPAT_OK;
}

void fill_info(qpat_info* info, const SolveStats& s) {
    if (!info) return;
    info->n_solves = s.n_solves;
    info->iters_max = s.iters_max;
    info->iters_sum = s.iters_sum;
    info->updates = s.updates;
    info->relres_max = s.relres_max;
    const int32_t n = std::min<int32_t>(std::max(info->rhs_cap, 0), static_cast<int32_t>(s.rhs_iters.size()));
    if (info->rhs_iters)
        for (int32_t i = 0; i < n; ++i) info->rhs_iters[i] = s.rhs_iters[i];
    if (info->rhs_relres)
        for (int32_t i = 0; i < n; ++i) info->rhs_relres[i] = s.rhs_relres[i];
}

qpat_status finish(qpat_ctx* c, const SolveStats& s, qpat_info* info) {
    fill_info(info, s);
    if (s.noconv)
        return fail(c, QPAT_ERR_NOCONV, "PCG did not reach the tolerance within pcg_maxit (relres %.3e)",
                    s.relres_max);
    return QPAT_OK;
}

qpat_status alloc_core(qpat_ctx* c) {
    const int64_t N = c->N, L = c->sell.len;
    QPAT_TRY(dalloc(c, &c->kappa, N));
    QPAT_TRY(dalloc(c, &c->mu, N));
    QPAT_TRY(dalloc(c, &c->K64, L));
    QPAT_TRY(dalloc(c, &c->K32, L));
    QPAT_TRY(dalloc(c, &c->Kdinv64, N));
    QPAT_TRY(dalloc(c, &c->Kdinv32, N));
    QPAT_TRY(dalloc(c, &c->M64, 2 * L));
    QPAT_TRY(dalloc(c, &c->M32, 2 * L));
    QPAT_TRY(dalloc(c, &c->Mdinv64, 2 * N));
    QPAT_TRY(dalloc(c, &c->Mdinv32, 2 * N));
    const int64_t V = N * kMaxRhs;  // >= 2N
    QPAT_TRY(dalloc(c, &c->x64, V));
    QPAT_TRY(dalloc(c, &c->b64, V));
    double* t = nullptr;
    QPAT_TRY(dalloc(c, &t, V)); c->xl = t;
    QPAT_TRY(dalloc(c, &t, V)); c->rl = t;
    QPAT_TRY(dalloc(c, &t, V)); c->pa = t;
    QPAT_TRY(dalloc(c, &t, V)); c->pb = t;
    QPAT_TRY(dalloc(c, &t, V)); c->ql = t;
    QPAT_TRY(dalloc(c, &c->scal, kMaxSys));
    QPAT_TRY(dalloc(c, &c->shared, 1));
    QPAT_HIP(c, hipMemsetAsync(c->shared, 0, sizeof(PcgShared), c->stream));
    QPAT_TRY(dalloc(c, &c->partials, (size_t)5 * kMaxSys * 2048));
    QPAT_TRY(dalloc(c, &c->acc1, N));
    QPAT_TRY(dalloc(c, &c->acc2, N));
    QPAT_TRY(dalloc(c, &c->red_partials, 1024));
    QPAT_TRY(dalloc(c, &c->red_out, 64));
    QPAT_TRY(dalloc(c, &c->red_counter, 16));
    QPAT_HIP(c, hipMemsetAsync(c->red_counter, 0, 16 * sizeof(uint32_t), c->stream));
    QPAT_TRY(dalloc(c, &c->ls, 1));
    QPAT_HIP(c, hipMemsetAsync(c->ls, 0, sizeof(LsqrScal), c->stream));
    QPAT_TRY(dalloc(c, &c->lv, 2 * N));
    QPAT_TRY(dalloc(c, &c->lwh, 2 * N));
    QPAT_TRY(dalloc(c, &c->lwd, 2 * N));
    QPAT_TRY(dalloc(c, &c->lp, 2 * N));
    QPAT_TRY(dalloc(c, &c->lr, 2 * N));
    QPAT_HIP(c, hipHostMalloc((void**)&c->scal_host, sizeof(PcgScal) * kMaxSys, hipHostMallocDefault));
    QPAT_HIP(c, hipHostMalloc((void**)&c->ls_host, sizeof(LsqrScal), hipHostMallocDefault));
    QPAT_HIP(c, hipHostMalloc((void**)&c->red_host, sizeof(double) * 64, hipHostMallocDefault));
    std::memset(c->ls_host, 0, sizeof(LsqrScal));
    return QPAT_OK;
}

qpat_status alloc_bases(qpat_ctx* c) {
    const int cap = c->opts.lsqr_max_steps + 1;
    if (c->basis_cap >= cap && c->U) return QPAT_OK;   // possibly grown by an earlier run
    QPAT_TRY(dfree(c, c->U));
    QPAT_TRY(dfree(c, c->V));
    QPAT_TRY(dfree(c, c->WH));
    QPAT_TRY(dfree(c, c->coef));
    c->U = c->V = c->WH = c->coef = nullptr;
    c->basis_cap = 0;
    QPAT_TRY(dalloc(c, &c->U, (size_t)cap * c->N * c->n_pad));
    QPAT_TRY(dalloc(c, &c->V, (size_t)cap * 2 * c->N));
    QPAT_TRY(dalloc(c, &c->WH, (size_t)cap * 2 * c->N));
    QPAT_TRY(dalloc(c, &c->coef, cap));
    c->basis_cap = cap;
    return QPAT_OK;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

}  // namespace
}  // namespace qpat

using namespace qpat;

extern "C" {

void qpat_default_opts(qpat_opts* o) {
    if (!o) return;
    o->precision = 0;
    o->max_rhs_block = 16;
    o->pcg_rtol = 1e-10;
    o->pcg_maxit = 20000;
    o->prior_rtol = 1e-8;
    o->prior_deflate = 1;
    o->lsqr_reorth = 1;
    o->lsqr_max_steps = 64;
    o->ru_delta = 1e-3;
    o->use_graphs = 1;
    o->operator_format = 1;
    o->prior_precond = 1;
    o->pcg_precond = 1;
    o->autotune = 1;
}

const char* qpat_version(void) { return "qpat 0.1 (gfx950)"; }

qpat_status qpat_setup_mesh(qpat_ctx** out, int64_t N, const double* coords, int64_t E, const int32_t* tets,
                            int64_t F_b, const int32_t* bfaces, const qpat_opts* opts, void* hip_stream) {
    if (!out) return QPAT_ERR_ARG;
    *out = nullptr;
    qpat_ctx* c = new (std::nothrow) qpat_ctx();
    if (!c) return QPAT_ERR_OOM;
    *out = c;
    if (!coords || !tets || N < 4 || E < 1 || F_b < 0 || (F_b > 0 && !bfaces))
        return fail(c, QPAT_ERR_ARG, "setup_mesh: bad sizes or null pointers");
    qpat_default_opts(&c->opts);
    if (opts) {
        QPAT_TRY(check_opts(c, opts));
        c->opts = *opts;
    }
    c->stream = static_cast<hipStream_t>(hip_stream);
    QPAT_HIP(c, hipGetDevice(&c->device));
    c->N = N;
    c->E = E;
    c->Fb = F_b;
    QPAT_TRY(scratch_setup(c));
    QPAT_TRY(mesh_build(c, coords, tets, bfaces));
    QPAT_TRY(alloc_core(c));
    QPAT_TRY(lattice_setup(c, coords));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_set_opts(qpat_ctx* c, const qpat_opts* o) {
    if (!c || !o) return QPAT_ERR_ARG;
    QPAT_TRY(check_opts(c, o));
    c->opts = *o;
    return QPAT_OK;
}

qpat_status qpat_get_opts(const qpat_ctx* c, qpat_opts* o) {
    if (!c || !o) return QPAT_ERR_ARG;
    *o = c->opts;
    return QPAT_OK;
}

qpat_status qpat_set_sources(qpat_ctx* c, int32_t n_ill, const double* phi_src) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (n_ill < 1 || n_ill > 64 || (!phi_src && c->Fb > 0))
        return fail(c, QPAT_ERR_ARG, "set_sources: need 1 <= n_ill <= 64 and a source array");
    int n_pad = 1;
    while (n_pad < n_ill && n_pad < kMaxRhs) n_pad <<= 1;
    if (n_ill > kMaxRhs) n_pad = ((n_ill + kMaxRhs - 1) / kMaxRhs) * kMaxRhs;
    if (n_pad != c->n_pad) {
        for (double** p : {&c->f, &c->phi, &c->dvec, &c->lu, &c->lq, &c->lw}) {
            QPAT_TRY(dfree(c, *p));
            *p = nullptr;
        }
        QPAT_TRY(dfree(c, c->U));
        QPAT_TRY(dfree(c, c->V));
        QPAT_TRY(dfree(c, c->WH));
        QPAT_TRY(dfree(c, c->coef));
        c->U = c->V = c->WH = c->coef = nullptr;
        c->basis_cap = 0;
        const int64_t nd = c->N * n_pad;
        for (double** p : {&c->f, &c->phi, &c->dvec, &c->lu, &c->lq, &c->lw}) QPAT_TRY(dalloc(c, p, nd));
    }
    c->n_ill = n_ill;
    c->n_pad = n_pad;
    c->have_forward = false;
    c->lsqr_ready = false;
    QPAT_TRY(assemble_load(c, phi_src));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

static qpat_status forward_common(qpat_ctx* c, double* phi_out, double* h_out, qpat_info* info,
                                  const double* x0 = nullptr) {
    QPAT_TRY(assemble_K(c));
    QPAT_TRY(lattice_convert(c, Op::K));
    QPAT_TRY(mg_setup(c, Op::K));
    SolveStats st;
    c->have_forward = false;
    c->lsqr_ready = false;
    if (x0) QPAT_TRY(forward_solve_x0(c, x0, &st));
    else QPAT_TRY(forward_solve(c, &st));
    const int64_t n = c->N * c->n_ill;
    const dim3 g(grid_for(n, kThreads, 1 << 30)), b(kThreads);
    if (phi_out) hipLaunchKernelGGL(k_from_interleaved, g, b, 0, c->stream, c->N, c->n_ill, c->n_pad, c->phi, nullptr, phi_out);
    if (h_out) hipLaunchKernelGGL(k_from_interleaved, g, b, 0, c->stream, c->N, c->n_ill, c->n_pad, c->phi, c->mu, h_out);
    QPAT_HIP(c, hipGetLastError());
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    qpat_status s = finish(c, st, info);
    if (s == QPAT_OK) c->have_forward = true;
    return s;
}

qpat_status qpat_forward(qpat_ctx* c, const double* kappa, const double* mu, double* phi_out, double* h_out,
                         qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!kappa || !mu) return fail(c, QPAT_ERR_ARG, "forward: null kappa or mu");
    if (c->n_ill == 0) return fail(c, QPAT_ERR_STATE, "forward: call qpat_set_sources first");
    bool ok1 = false, ok2 = false;
    QPAT_TRY(check_positive(c, kappa, c->N, &ok1));
    QPAT_TRY(check_positive(c, mu, c->N, &ok2));
    if (!ok1 || !ok2) return fail(c, QPAT_ERR_ARG, "forward: kappa and mu must be finite and > 0");
    const dim3 gr(grid_for(c->N, kThreads, 1 << 30)), b(kThreads);
    hipLaunchKernelGGL(k_copy_d, gr, b, 0, c->stream, c->N, kappa, c->kappa);
    hipLaunchKernelGGL(k_copy_d, gr, b, 0, c->stream, c->N, mu, c->mu);
    return forward_common(c, phi_out, h_out, info);
}

qpat_status qpat_forward_x0(qpat_ctx* c, const double* kappa, const double* mu, const double* x0,
                            double* phi_out, double* h_out, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!kappa || !mu || !x0) return fail(c, QPAT_ERR_ARG, "forward_x0: null pointer");
    if (c->n_ill == 0) return fail(c, QPAT_ERR_STATE, "forward_x0: call qpat_set_sources first");
    bool ok1 = false, ok2 = false;
    QPAT_TRY(check_positive(c, kappa, c->N, &ok1));
    QPAT_TRY(check_positive(c, mu, c->N, &ok2));
    if (!ok1 || !ok2) return fail(c, QPAT_ERR_ARG, "forward_x0: kappa and mu must be finite and > 0");
    const dim3 gr(grid_for(c->N, kThreads, 1 << 30)), b(kThreads);
    hipLaunchKernelGGL(k_copy_d, gr, b, 0, c->stream, c->N, kappa, c->kappa);
    hipLaunchKernelGGL(k_copy_d, gr, b, 0, c->stream, c->N, mu, c->mu);
    return forward_common(c, phi_out, h_out, info, x0);
}

qpat_status qpat_guess_setup(qpat_ctx* c, int32_t nx, int32_t ny, int32_t nz) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (nx < 1 || ny < 1 || nz < 1) return fail(c, QPAT_ERR_ARG, "guess_setup: bad lattice");
    QPAT_TRY(guess_setup(c, nx, ny, nz));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

#define QPAT_NEED_GUESS(c)                                                                 \
    do {                                                                                   \
        if (!(c)->guess) return fail((c), QPAT_ERR_STATE, "call qpat_guess_setup first"); \
    } while (0)

qpat_status qpat_guess_set_params(qpat_ctx* c, const float* params) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!params) return fail(c, QPAT_ERR_ARG, "guess_set_params: null pointer");
    QPAT_TRY(guess_set_params(c, params));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_guess_get_params(qpat_ctx* c, float* params) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!params) return fail(c, QPAT_ERR_ARG, "guess_get_params: null pointer");
    QPAT_TRY(guess_get_params(c, params));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_guess_eval(qpat_ctx* c, const float* input, float* out) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!input || !out) return fail(c, QPAT_ERR_ARG, "guess_eval: null pointer");
    QPAT_TRY(guess_eval_raw(c, input, out));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_guess_grad(qpat_ctx* c, const float* input, const float* target, float* grad, double* loss) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!input || !target) return fail(c, QPAT_ERR_ARG, "guess_grad: null pointer");
    return guess_grad_raw(c, input, target, grad, loss);
}

qpat_status qpat_guess_train_step(qpat_ctx* c, const float* input, const float* target, float lr, double* loss) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!input || !target || !(lr > 0.f)) return fail(c, QPAT_ERR_ARG, "guess_train_step: bad arguments");
    QPAT_TRY(guess_train_raw(c, input, target, lr, loss));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_guess_train(qpat_ctx* c, const double* kappa, const double* mu, double kappa0, double mu0,
                             const double* phi_hom, const double* phi, float lr, double* loss) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!kappa || !mu || !phi_hom || !phi || !(lr > 0.f) || !(kappa0 > 0) || !(mu0 > 0))
        return fail(c, QPAT_ERR_ARG, "guess_train: bad arguments");
    return guess_train(c, kappa, mu, kappa0, mu0, phi_hom, phi, lr, loss);
}

qpat_status qpat_guess_fluence(qpat_ctx* c, const double* kappa, const double* mu, double kappa0, double mu0,
                               const double* phi_hom, double* phi0_out) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    QPAT_NEED_GUESS(c);
    if (!kappa || !mu || !phi_hom || !phi0_out || !(kappa0 > 0) || !(mu0 > 0))
        return fail(c, QPAT_ERR_ARG, "guess_fluence: bad arguments");
    if (c->n_ill == 0) return fail(c, QPAT_ERR_STATE, "guess_fluence: call qpat_set_sources first");
    QPAT_TRY(guess_fluence(c, kappa, mu, kappa0, mu0, phi_hom, phi0_out));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_forward_log(qpat_ctx* c, double kappa0, double mu0, const double* beta, double* phi_out,
                             double* h_out, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!beta || !(kappa0 > 0.0) || !(mu0 > 0.0)) return fail(c, QPAT_ERR_ARG, "forward_log: bad arguments");
    if (c->n_ill == 0) return fail(c, QPAT_ERR_STATE, "forward_log: call qpat_set_sources first");
    QPAT_TRY(exp_params(c, kappa0, mu0, beta));
    bool ok1 = false, ok2 = false;
    QPAT_TRY(check_positive(c, c->kappa, c->N, &ok1));
    QPAT_TRY(check_positive(c, c->mu, c->N, &ok2));
    if (!ok1 || !ok2) return fail(c, QPAT_ERR_ARG, "forward_log: exp(beta) not finite and positive");
    return forward_common(c, phi_out, h_out, info);
}

qpat_status qpat_jvp(qpat_ctx* c, const double* s, double* out, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!s || !out) return fail(c, QPAT_ERR_ARG, "jvp: null pointer");
    if (!c->have_forward) return fail(c, QPAT_ERR_STATE, "jvp: call qpat_forward first");
    SolveStats st;
    QPAT_TRY(jvp_core(c, s, 0, out, &st));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return finish(c, st, info);
}

qpat_status qpat_vjp(qpat_ctx* c, const double* t, double* out, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!t || !out) return fail(c, QPAT_ERR_ARG, "vjp: null pointer");
    if (!c->have_forward) return fail(c, QPAT_ERR_STATE, "vjp: call qpat_forward first");
    SolveStats st;
    QPAT_TRY(vjp_core(c, t, 0, out, &st));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return finish(c, st, info);
}

qpat_status qpat_prior_setup(qpat_ctx* c, const double* kt, const double* mt, double T, double b_over_a,
                             double delta) {
    return qpat_prior_setup_r(c, kt, mt, QPAT_PRIOR_PM, T, 1.0, b_over_a, delta);
}

qpat_status qpat_prior_setup_r(qpat_ctx* c, const double* kt, const double* mt, int32_t kind, double T, double q,
                               double b_over_a, double delta) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!kt || !mt || !(T > 0.0) || !(b_over_a > 0.0) || !(delta > 0.0))
        return fail(c, QPAT_ERR_ARG, "prior_setup: need kt, mt and T, b_over_a, delta > 0");
    if (kind != QPAT_PRIOR_PM && kind != QPAT_PRIOR_TVQ)
        return fail(c, QPAT_ERR_ARG, "prior_setup: unknown prior kind %d", (int)kind);
    if (kind == QPAT_PRIOR_TVQ && !(q > 0.0 && q <= 2.0))
        return fail(c, QPAT_ERR_ARG, "prior_setup: TV^q needs 0 < q <= 2");
    QPAT_TRY(assemble_prior(c, kt, mt, kind, T, q, b_over_a, delta));
    QPAT_TRY(lattice_convert(c, Op::Prior));
    c->delta = delta;
    QPAT_TRY(mg_setup(c, Op::Prior));
    c->have_prior = true;
    c->lsqr_ready = false;
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_prior_apply(qpat_ctx* c, const double* x, double* y) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!x || !y) return fail(c, QPAT_ERR_ARG, "prior_apply: null pointer");
    if (!c->have_prior) return fail(c, QPAT_ERR_STATE, "prior_apply: call qpat_prior_setup first");
    QPAT_TRY(prior_apply_core(c, x, y));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

qpat_status qpat_prior_solve(qpat_ctx* c, const double* p, double* r, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!p || !r) return fail(c, QPAT_ERR_ARG, "prior_solve: null pointer");
    if (!c->have_prior) return fail(c, QPAT_ERR_STATE, "prior_solve: call qpat_prior_setup first");
    SolveStats st;
    QPAT_TRY(prior_solve_core(c, p, r, &st));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return finish(c, st, info);
}

qpat_status qpat_misfit(qpat_ctx* c, const double* chi, const double* w, double* out) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!chi || !w || !out) return fail(c, QPAT_ERR_ARG, "misfit: null pointer");
    if (!c->have_forward) return fail(c, QPAT_ERR_STATE, "misfit: call qpat_forward first");
    return misfit_core(c, chi, w, out);
}

qpat_status qpat_misfit_noalloc(qpat_ctx* c, const double* chi, const double* w, double* out_dev) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!chi || !w || !out_dev) return fail(c, QPAT_ERR_ARG, "misfit_noalloc: null pointer");
    if (!c->have_forward) return fail(c, QPAT_ERR_STATE, "misfit_noalloc: call qpat_forward first");
    return misfit_noalloc_core(c, chi, w, out_dev);
}

qpat_status qpat_init_guess(qpat_ctx* c, const double* chi, double mu0, double* beta_out) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!chi || !beta_out || !(mu0 > 0.0)) return fail(c, QPAT_ERR_ARG, "init_guess: bad arguments");
    if (!c->have_forward) return fail(c, QPAT_ERR_STATE, "init_guess: call qpat_forward first");
    QPAT_TRY(init_guess_core(c, chi, mu0, beta_out));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

static qpat_status lsqr_init_common(qpat_ctx* c, const double* chi, const double* w, const double* beta_lin,
                                    double* beta_out, qpat_info* info, bool kappa_only) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!chi || !w || !beta_out) return fail(c, QPAT_ERR_ARG, "lsqr_init: null pointer");
    if (!c->have_forward || !c->have_prior)
        return fail(c, QPAT_ERR_STATE, "lsqr_init: needs qpat_forward and qpat_prior_setup");
    c->lsqr_ready = false;
    c->ls_kappa_only = kappa_only;
    if (c->opts.lsqr_reorth) QPAT_TRY(alloc_bases(c));
    c->lx = beta_out;
    QPAT_TRY(lsqr_init_core(c, chi, w, beta_lin));
    c->lsqr_ready = true;
    fill_info(info, SolveStats());
    return QPAT_OK;
}

qpat_status qpat_lsqr_init(qpat_ctx* c, const double* chi, const double* w, const double* beta_lin,
                           double* beta_out, qpat_info* info) {
    return lsqr_init_common(c, chi, w, beta_lin, beta_out, info, false);
}

qpat_status qpat_lsqr_init_kappa(qpat_ctx* c, const double* chi, const double* w, const double* beta_lin,
                                 double* beta_out, qpat_info* info) {
    return lsqr_init_common(c, chi, w, beta_lin, beta_out, info, true);
}

// Background fit of Algorithm 1's preamble: (log kappa, log mu) by Gauss-Newton
// on |W (chi - h(kappa 1, mu 1))|^2. The two Jacobian columns are J [1; 0] and
// J [0; 1] at the current homogeneous point (d/dlog kappa = kappa d/dkappa).
// A step longer than 1 in either log is shortened to 1, and halved (up to 30
// times) until the misfit does not increase; the fit stops when the accepted
// step is at most tol in both logs, or when no halving decreases the misfit.
qpat_status qpat_fit_background(qpat_ctx* c, const double* chi, const double* w, double* kappa0, double* mu0,
                                int32_t maxit, double tol, int32_t* iters, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!chi || !w || !kappa0 || !mu0 || !(*kappa0 > 0.0) || !(*mu0 > 0.0) || !std::isfinite(*kappa0) ||
        !std::isfinite(*mu0) || maxit < 0 || !(tol >= 0.0))
        return fail(c, QPAT_ERR_ARG, "fit_background: need chi, w, finite kappa0, mu0 > 0, maxit >= 0, tol >= 0");
    if (c->n_ill == 0) return fail(c, QPAT_ERR_STATE, "fit_background: call qpat_set_sources first");
    const int64_t N = c->N, nd = N * c->n_ill;
    double *zero = nullptr, *s1 = nullptr, *s2 = nullptr, *j1 = nullptr, *j2 = nullptr, *rr = nullptr;
    auto release = [&]() {
        for (double* p : {zero, s1, s2, j1, j2, rr})
            if (p) (void)dfree(c, p);
    };
    struct Guard {
        std::function<void()> f;
        ~Guard() { f(); }
    } guard{release};
    QPAT_TRY(dalloc(c, &zero, 2 * N));
    QPAT_TRY(dalloc(c, &s1, 2 * N));
    QPAT_TRY(dalloc(c, &s2, 2 * N));
    QPAT_TRY(dalloc(c, &j1, nd));
    QPAT_TRY(dalloc(c, &j2, nd));
    QPAT_TRY(dalloc(c, &rr, nd));
    QPAT_TRY(zero_fill(c, zero, 2 * N));
    QPAT_TRY(zero_fill(c, s1 + N, N));
    QPAT_TRY(zero_fill(c, s2, N));
    QPAT_TRY(exp_params(c, 1.0, 1.0, zero));   // kappa = mu = 1: the all-ones halves of s1, s2
    QPAT_HIP(c, hipMemcpyAsync(s1, c->kappa, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    QPAT_HIP(c, hipMemcpyAsync(s2 + N, c->mu, N * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    SolveStats st;
    c->have_forward = false;
    c->lsqr_ready = false;
    // misfit^2 at the homogeneous point (exp a, exp b); leaves the forward state there
    auto evaluate = [&](double a, double b, double* F) -> qpat_status {
        const double k = std::exp(a), m = std::exp(b);
        if (!(k > 0.0) || !(m > 0.0) || !std::isfinite(k) || !std::isfinite(m))
            return fail(c, QPAT_ERR_BREAKDOWN, "fit_background: the iterate left the positive reals");
        c->have_forward = false;
        QPAT_TRY(exp_params(c, k, m, zero));
        QPAT_TRY(assemble_K(c));
        QPAT_TRY(lattice_convert(c, Op::K));
        QPAT_TRY(mg_setup(c, Op::K));
        QPAT_TRY(forward_solve(c, &st));
        if (st.noconv)
            return fail(c, QPAT_ERR_NOCONV, "fit_background: PCG did not converge (relres %.3e)", st.relres_max);
        c->have_forward = true;
        double r = 0.0;
        QPAT_TRY(misfit_core(c, chi, w, &r));
        *F = r * r;
        return QPAT_OK;
    };
    double a = std::log(*kappa0), b = std::log(*mu0), F = 0.0;
    QPAT_TRY(evaluate(a, b, &F));
    int it = 0;
    bool at_ab = true;
    for (; it < maxit; ++it) {
        SolveStats sj;
        QPAT_TRY(jvp_core(c, s1, 0, j1, &sj));
        QPAT_TRY(jvp_core(c, s2, 0, j2, &sj));
        if (sj.noconv) return fail(c, QPAT_ERR_NOCONV, "fit_background: PCG did not converge in J");
        st.merge(sj);
        double S[6];
        QPAT_TRY(fit_sums(c, chi, w, j1, j2, rr, S));
        const double det = S[0] * S[2] - S[1] * S[1];
        if (!(det > 0.0) || !std::isfinite(det))
            return fail(c, QPAT_ERR_BREAKDOWN, "fit_background: singular Gauss-Newton matrix");
        double da = (S[2] * S[3] - S[1] * S[4]) / det, db = (S[0] * S[4] - S[1] * S[3]) / det;
        const double len = std::max(std::fabs(da), std::fabs(db));
        if (len > 1.0) {
            da /= len;
            db /= len;
        }
        double t = 1.0, Fn = 0.0;
        bool accepted = false;
        for (int h = 0; h <= 30; ++h, t *= 0.5) {
            QPAT_TRY(evaluate(a + t * da, b + t * db, &Fn));
            if (Fn <= F) {
                accepted = true;
                break;
            }
        }
        if (!accepted) {
            at_ab = false;
            break;
        }
        a += t * da;
        b += t * db;
        F = Fn;
        if (std::max(std::fabs(t * da), std::fabs(t * db)) <= tol) {
            ++it;
            break;
        }
    }
    if (!at_ab) QPAT_TRY(evaluate(a, b, &F));   // leave the forward state at the returned point
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    if (it > 0) {   // with no accepted step the caller's pair is returned as given
        *kappa0 = std::exp(a);
        *mu0 = std::exp(b);
    }
    if (iters) *iters = it;
    fill_info(info, st);
    return QPAT_OK;
}

qpat_status qpat_lsqr_step(qpat_ctx* c, double* resnorm_out, qpat_info* info) {
    if (!c) return QPAT_ERR_ARG;
    DeviceGuard g(c->device);
    if (!c->lsqr_ready) return fail(c, QPAT_ERR_STATE, "lsqr_step: call qpat_lsqr_init first");
    SolveStats st;
    QPAT_TRY(lsqr_step_core(c, &st));
    if (resnorm_out) *resnorm_out = std::fabs(c->ls_host->phibar);
    return finish(c, st, info);
}

qpat_status qpat_batch(qpat_ctx* const* ctxs, int32_t n, int32_t op, const double* const* in0, double* const* out0,
                       const double* const* in1, double* const* out1, qpat_info* infos) {
    if (!ctxs || n < 1 || n > 256 || op < QPAT_BATCH_FORWARD || op > QPAT_BATCH_LSQR_STEP) return QPAT_ERR_ARG;
    for (int i = 0; i < n; ++i) {
        if (!ctxs[i]) return QPAT_ERR_ARG;
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == ctxs[i] || ctxs[j]->stream == ctxs[i]->stream)
                return fail(ctxs[i], QPAT_ERR_ARG, "batch: contexts %d and %d share a context or a stream", j, i);
        const bool need0 = op != QPAT_BATCH_LSQR_STEP, need1 = op == QPAT_BATCH_FORWARD || op == QPAT_BATCH_PAIR;
        if ((need0 && (!in0 || !in0[i])) || (need1 && (!in1 || !in1[i])) ||
            ((op == QPAT_BATCH_JVP || op == QPAT_BATCH_VJP || op == QPAT_BATCH_PAIR) && (!out0 || !out0[i])) ||
            (op == QPAT_BATCH_PAIR && (!out1 || !out1[i])))
            return fail(ctxs[i], QPAT_ERR_ARG, "batch: missing array for instance %d", i);
    }
    std::vector<qpat_status> st(n, QPAT_OK);
    std::vector<qpat_info> inf(n);
    auto work = [&](int i) {
        qpat_ctx* c = ctxs[i];
        // the caller's per-right-hand-side arrays (if any) are kept; the pair's
        // second call continues where the first stopped
        qpat_info a{}, b{};
        if (infos) {
            a.rhs_cap = infos[i].rhs_cap;
            a.rhs_iters = infos[i].rhs_iters;
            a.rhs_relres = infos[i].rhs_relres;
        }
        switch (op) {
            case QPAT_BATCH_FORWARD:
                st[i] = qpat_forward(c, in0[i], in1[i], nullptr, out0 ? out0[i] : nullptr, &a);
                break;
            case QPAT_BATCH_JVP: st[i] = qpat_jvp(c, in0[i], out0[i], &a); break;
            case QPAT_BATCH_VJP: st[i] = qpat_vjp(c, in0[i], out0[i], &a); break;
            case QPAT_BATCH_PAIR:
                st[i] = qpat_jvp(c, in0[i], out0[i], &a);
                if (a.rhs_cap > a.n_solves) {
                    b.rhs_cap = a.rhs_cap - a.n_solves;
                    b.rhs_iters = a.rhs_iters ? a.rhs_iters + a.n_solves : nullptr;
                    b.rhs_relres = a.rhs_relres ? a.rhs_relres + a.n_solves : nullptr;
                }
                if (st[i] == QPAT_OK) st[i] = qpat_vjp(c, in1[i], out1[i], &b);
                a.n_solves += b.n_solves;
                a.iters_max = std::max(a.iters_max, b.iters_max);
                a.iters_sum += b.iters_sum;
                a.updates += b.updates;
                a.relres_max = std::max(a.relres_max, b.relres_max);
                break;
            default: st[i] = qpat_lsqr_step(c, nullptr, &a); break;
        }
        inf[i] = a;
    };
    std::vector<std::thread> pool;
    pool.reserve(n - 1);
    for (int i = 1; i < n; ++i) pool.emplace_back(work, i);
    work(0);
    for (auto& t : pool) t.join();
    if (infos)
        for (int i = 0; i < n; ++i) infos[i] = inf[i];
    for (int i = 0; i < n; ++i)
        if (st[i] != QPAT_OK) return st[i];
    return QPAT_OK;
}

qpat_status qpat_profile(qpat_ctx* c, int32_t enable) {
    if (!c) return QPAT_ERR_ARG;
    if (enable) {
        for (auto& k : c->prof) k = qpat_kstat{0, 0, 0.0, 0.0, 0.0};
    }
    c->prof_on = enable != 0;
    return QPAT_OK;
}

qpat_status qpat_profile_read(const qpat_ctx* c, qpat_kstat out[QPAT_NKSTAT]) {
    if (!c || !out) return QPAT_ERR_ARG;
    for (int i = 0; i < QPAT_NKSTAT; ++i) out[i] = c->prof[i];
    return QPAT_OK;
}

qpat_status qpat_operator_layout(const qpat_ctx* c, int64_t out[6]) {
    if (!c || !out) return QPAT_ERR_ARG;
    out[0] = c->lat.on ? 1 : 0;
    out[1] = c->lat.nx;
    out[2] = c->lat.ny;
    out[3] = c->lat.nz;
    out[4] = c->lat.on ? c->lat.m + 1 : 0;
    out[5] = c->sell.len;
    return QPAT_OK;
}

qpat_status qpat_tile_schedule(const qpat_ctx* c, int32_t B, int32_t out[8]) {
    if (!c || !out || (B != 8 && B != 16)) return QPAT_ERR_ARG;
    return mg_tile_schedule(c, B, out);
}

int32_t qpat_geometry_classes(const qpat_ctx* c) { return c ? c->geo_ncls : -1; }

int32_t qpat_lsqr_steps(const qpat_ctx* c) { return c && c->ls_host ? c->ls_host->steps : 0; }

int32_t qpat_lsqr_basis(const qpat_ctx* c) { return c && c->reorth_on ? c->nbasis : 0; }

double qpat_lsqr_residual(const qpat_ctx* c) {
    if (!c || !c->ls_host || !c->lsqr_ready) return -1.0;
    return std::fabs(c->ls_host->phibar);
}

const char* qpat_last_error(const qpat_ctx* c) { return c ? c->err.c_str() : "null context"; }

void qpat_destroy(qpat_ctx* c) {
    if (!c) return;
    DeviceGuard g(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    guess_destroy(c);
    mg_destroy(c);
    for (void* p : c->allocs) (void)hipFree(p);
    c->allocs.clear();
    if (c->scal_host) (void)hipHostFree(c->scal_host);
    if (c->ls_host) (void)hipHostFree(c->ls_host);
    if (c->red_host) (void)hipHostFree(c->red_host);
    delete c;
}

}  // extern "C"
