// Priorconditioned LSQR (Sec. 4 eq. (4.10); Algorithm 1 step 3) with FP64
// recurrences on the device, plus the prior apply/solve wrappers, the
// whitened misfit and the initial guess of Algorithm 1.
//
// Paige-Saunders LSQR applied to Abar = A L^{-1}, M_delta = L^T L, written in
// v = L^{-1} vbar, w = L^{-1} wbar, x = L^{-1} xbar and what = M_delta v so that
// only M_delta^{-1} is needed:
//   beta_1 u = yt;  p = A^T u;  r = M_delta^{-1} p;  alpha = sqrt(p.r);  v = r/alpha;  what = p/alpha
//   step: q = A v - alpha u; beta = |q|; u = q/beta
//         p = A^T u - beta what; r = M_delta^{-1} p; alpha = sqrt(p.r); v = r/alpha; what = p/alpha
//         rho = hypot(rhobar, beta); c = rhobar/rho; s = beta/rho; theta = s alpha
//         rhobar = -c alpha; phi = c phibar; phibar = s phibar
//         x += (phi/rho) w; w = v - (theta/rho) w
// Optional full reorthogonalisation (classical Gram-Schmidt, two passes): q
// against the stored u_j, and p against vbar_j = L v_j in the form
// p -= (v_j . p) what_j. Every dot product is a deterministic two-stage
// reduction; every scalar stays on the device.
// Dot products are two kernels: per-block partial sums, then one block adds
// them in a fixed order.
#include <cmath>
#include <mutex>

#include "qpat_internal.h"

namespace qpat {
namespace {

constexpr int kRedBlocks = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__device__ double block_total(double v) {
    __shared__ double sm[kThreads / 64];
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kThreads / 64; ++w) t += sm[w];
    __syncthreads();
    return t;
}

// partials[block] = sum of f(i) over the block's contiguous chunk of [0, n)
template <typename F>
__device__ void block_partials(F f, int64_t n, double* partials) {
    const int64_t chunk = (n + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = blockIdx.x * chunk;
    int64_t b1 = b0 + chunk;
    if (b1 > n) b1 = n;
    double a0 = 0.0, a1 = 0.0;
    int64_t i = b0 + threadIdx.x;
    for (; i + kThreads < b1; i += 2 * kThreads) {
        a0 += f(i);
        a1 += f(i + kThreads);
    }
    if (i < b1) a0 += f(i);
    const double t = block_total(a0 + a1);
    if (threadIdx.x == 0) partials[blockIdx.x] = t;
}

// out = sum of nb partials in a fixed order (one block)
__global__ __launch_bounds__(kThreads) void k_sum_partials(const double* __restrict__ partials, int nb,
                                                           double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += partials[b];
    s = block_total(s);
    if (threadIdx.x == 0) *out = s;
}

__global__ __launch_bounds__(kThreads) void k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t n, double* partials) {
    block_partials([=] __device__(int64_t i) { return a[i] * b[i]; }, n, partials);
}

// ||W (chi - mu phi)||^2 with chi, W external [n_ill][N], phi interleaved
__global__ __launch_bounds__(kThreads) void k_misfit(int64_t N, int n_ill, int n_pad, const double* __restrict__ chi,
                                                     const double* __restrict__ w, const double* __restrict__ mu,
                                                     const double* __restrict__ phi, double* partials) {
    block_partials(
        [=] __device__(int64_t i) {
            const int64_t k = i / N, row = i % N;
            const double d = w[i] * (chi[i] - mu[row] * phi[row * n_pad + k]);
            return d * d;
        },
        N * n_ill, partials);
}

// u = W (chi - mu phi + Jb), interleaved; Jb interleaved (or null); also W interleaved
__global__ void k_lsqr_rhs(int64_t N, int n_ill, int n_pad, const double* __restrict__ chi,
                           const double* __restrict__ w, const double* __restrict__ mu,
                           const double* __restrict__ phi, const double* __restrict__ Jb, double* __restrict__ u,
                           double* __restrict__ Wi) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * n_pad) return;
    const int64_t row = t / n_pad;
    const int k = static_cast<int>(t % n_pad);
    if (k >= n_ill) {
        u[t] = 0.0;
        Wi[t] = 0.0;
        return;
    }
    const int64_t e = (int64_t)k * N + row;
    double y = chi[e] - mu[row] * phi[t];
    if (Jb) y += Jb[t];
    u[t] = w[e] * y;
    Wi[t] = w[e];
}

// ---- scalar recurrences (single thread)
// init: beta1 = sqrt(uu); u is scaled later by 1/beta1
__global__ void k_ls_init_beta(LsqrScal* ls, const double* uu) {
    if (threadIdx.x != 0) return;
    const double b = sqrt(*uu);
    ls->beta1 = b;
    ls->phibar = b;
    ls->beta = b;
    ls->done = b == 0.0 || !(b == b);
    ls->breakdown = !(b == b);
    ls->steps = 0;
    ls->rotated = 0;
    ls->alpha = 0.0;
    ls->rhobar = 0.0;
}

__global__ void k_ls_init_alpha(LsqrScal* ls, const double* pr) {
    if (threadIdx.x != 0 || ls->done) return;
    const double v = *pr;
    if (!(v >= 0.0) || !(v < INFINITY)) {
        ls->breakdown = 1;
        ls->done = 1;
        return;
    }
    ls->alpha = sqrt(v);
    ls->rhobar = ls->alpha;
    if (ls->alpha == 0.0) ls->done = 1;
}

// after q (= A v - alpha u, reorthogonalised): beta = |q|
__global__ void k_ls_beta(LsqrScal* ls, const double* qq) {
    if (threadIdx.x != 0 || ls->done) return;
    const double b = sqrt(*qq);
    ls->beta = b;
    ls->rotated = 0;
    if (!(b == b)) {
        ls->breakdown = 1;
        ls->done = 1;
    }
}

// after p, r: alpha and the plane rotation
__global__ void k_ls_rotate(LsqrScal* ls, const double* pr) {
    if (threadIdx.x != 0 || ls->done) return;
    const double v = *pr;
    if (!(v >= 0.0) || !(v < INFINITY)) {
        ls->breakdown = 1;
        ls->done = 1;
        return;
    }
    const double alpha = sqrt(v);
    const double rho = hypot(ls->rhobar, ls->beta);
    const double c = ls->rhobar / rho, s = ls->beta / rho;
    ls->rho = rho;
    ls->c = c;
    ls->s = s;
    ls->theta = s * alpha;
    ls->rhobar = -c * alpha;
    ls->phi = c * ls->phibar;
    ls->phibar = s * ls->phibar;
    ls->alpha = alpha;
    ls->steps += 1;
    ls->rotated = 1;
}

// lucky breakdown beta = 0: x += (phibar/rhobar) w, stop
__global__ void k_ls_lucky(LsqrScal* ls, int64_t n2, double* __restrict__ x, const double* __restrict__ w) {
    if (ls->done || ls->beta != 0.0) return;
    const double f = ls->phibar / ls->rhobar;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x)
        x[i] += f * w[i];
}

__global__ void k_ls_lucky_flag(LsqrScal* ls) {
    if (threadIdx.x == 0 && !ls->done && ls->beta == 0.0) {
        ls->phibar = 0.0;
        ls->done = 1;
        ls->steps += 1;
    }
}

// u = q / beta (skip when done)
__global__ void k_ls_scale_u(const LsqrScal* ls, int64_t n, const double* __restrict__ q, double* __restrict__ u,
                             int use_beta1) {
    if (ls->done && !use_beta1) return;
    const double b = use_beta1 ? ls->beta1 : ls->beta;
    if (!(b > 0.0)) return;
    const double inv = 1.0 / b;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        u[i] = q[i] * inv;
}

// v = r/alpha, what = p/alpha, w = v (init)
__global__ void k_ls_first_v(const LsqrScal* ls, int64_t n2, const double* __restrict__ r,
                             const double* __restrict__ p, double* __restrict__ v, double* __restrict__ wh,
                             double* __restrict__ w, double* __restrict__ x) {
    const bool ok = !ls->done && ls->alpha > 0.0;
    const double inv = ok ? 1.0 / ls->alpha : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const double vi = r[i] * inv;
        v[i] = vi;
        wh[i] = p[i] * inv;
        w[i] = vi;
        x[i] = 0.0;
    }
}

// x += (phi/rho) w; v = r/alpha; what = p/alpha; w = v - (theta/rho) w
__global__ void k_ls_update(const LsqrScal* ls, int64_t n2, const double* __restrict__ r,
                            const double* __restrict__ p, double* __restrict__ v, double* __restrict__ wh,
                            double* __restrict__ w, double* __restrict__ x) {
    if (!ls->rotated) return;  // no rotation this step (lucky breakdown, breakdown)
    const double fx = ls->phi / ls->rho;
    const double ft = ls->theta / ls->rho;
    const double inv = ls->alpha > 0.0 ? 1.0 / ls->alpha : 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n2; i += (int64_t)gridDim.x * blockDim.x) {
        const double wi = w[i];
        x[i] += fx * wi;
        const double vi = r[i] * inv;
        v[i] = vi;
        wh[i] = p[i] * inv;
        w[i] = vi - ft * wi;
    }
}

__global__ void k_ls_alpha_zero(LsqrScal* ls) {
    if (threadIdx.x == 0 && ls->rotated && ls->alpha == 0.0) ls->done = 1;
}

// y -= sum_j coef[j] B_j  (B_j strided by ld)
__global__ void k_sub_combo(int64_t n, int nb, const double* __restrict__ coef, const double* __restrict__ Bm,
                            int64_t ld, double* __restrict__ y, const LsqrScal* ls) {
    if (ls->done) return;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = 0; j < nb; ++j) s += coef[j] * Bm[j * ld + i];
        y[i] -= s;
    }
}

__global__ void k_copy(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        b[i] = a[i];
}

// prior solve output: r = x + mean_s (mean = mean(p_s)/delta for deflated runs, else 0)
__global__ void k_prior_out(int64_t N, const double* __restrict__ x, const PcgScal* __restrict__ sc,
                            double* __restrict__ r) {
    const int sys = blockIdx.y;
    const double m = sc[sys].mean;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        r[sys * N + i] = x[sys * N + i] + m;
}

__global__ void k_init_guess(int64_t N, int n_ill, int n_pad, const double* __restrict__ chi,
                             const double* __restrict__ phi, double mu0, double* __restrict__ beta) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double s = 0.0;
    for (int k = 0; k < n_ill; ++k) s += chi[(int64_t)k * N + i] / phi[i * n_pad + k];
    double m = s / n_ill;
    if (!(m >= 1e-12 * mu0)) m = 1e-12 * mu0;
    beta[i] = 0.0;
    beta[N + i] = log(m / mu0);
}

inline dim3 grid1(int64_t n) { return dim3(grid_for(n, kThreads, 8192)); }

// background fit: rr = W (chi - mu phi) and j1, j2 scaled by W, all [n_ill][N]
__global__ void k_fit_weight(int64_t N, int n_ill, int n_pad, const double* __restrict__ chi,
                             const double* __restrict__ w, const double* __restrict__ mu,
                             const double* __restrict__ phi, double* __restrict__ j1, double* __restrict__ j2,
                             double* __restrict__ rr) {
    const int64_t n = N * n_ill;
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
        const int64_t i = e % N;
        const int k = static_cast<int>(e / N);
        const double we = w[e];
        rr[e] = we * (chi[e] - mu[i] * phi[i * n_pad + k]);
        j1[e] *= we;
        j2[e] *= we;
    }
}

__global__ void k_fill0(int64_t n, double* __restrict__ p) {
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads)
        p[e] = 0.0;
}

}  // namespace

qpat_status zero_fill(qpat_ctx* c, double* p, int64_t n) {
    hipLaunchKernelGGL(k_fill0, grid1(n), dim3(kThreads), 0, c->stream, n, p);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status fit_sums(qpat_ctx* c, const double* chi, const double* w, double* j1, double* j2, double* rr,
                     double out[6]) {
    const int64_t n = c->N * c->n_ill;
    hipLaunchKernelGGL(k_fit_weight, grid1(n), dim3(kThreads), 0, c->stream, c->N, c->n_ill, c->n_pad, chi, w,
                       c->mu, c->phi, j1, j2, rr);
    const double* a[6] = {j1, j1, j2, j1, j2, rr};
    const double* b[6] = {j1, j2, j2, rr, rr, rr};
    for (int q = 0; q < 6; ++q) QPAT_TRY(dot(c, a[q], b[q], n, c->red_out + 16 + q));
    QPAT_HIP(c, hipMemcpyAsync(c->red_host + 16, c->red_out + 16, 6 * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    for (int q = 0; q < 6; ++q) out[q] = c->red_host[16 + q];
    return QPAT_OK;
}

qpat_status dot(qpat_ctx* c, const double* a, const double* b, int64_t n, double* dev_out) {
    const int nb = grid_for(n, kThreads * 8, kRedBlocks);
    hipLaunchKernelGGL(k_dot, dim3(nb), dim3(kThreads), 0, c->stream, a, b, n, c->red_partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, c->stream, c->red_partials, nb, dev_out);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// ---- allocation-free misfit
// The partial sums of qpat_misfit_noalloc live in a file-scope device array
// (one copy per GPU, held until the process ends) instead of the context's
// workspace. The grid of k_misfit is capped at kRedBlocks blocks (each sums a
// contiguous chunk), so kRedBlocks partials cover every problem size. In host
// code `scratch` is only a stand-in for the symbol: its device address comes
// from hipGetSymbolAddress, looked up once per device.
static __device__ __align__(256) double scratch[kRedBlocks];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

__global__ __launch_bounds__(kThreads) void k_sum_sqrt(const double* __restrict__ partials, int nb,
                                                       double* __restrict__ out) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) s += partials[b];
    s = block_total(s);
    if (threadIdx.x == 0) *out = sqrt(s);
}

}  // namespace

// Device address of this GPU's scratch array; the context's device must be current.
qpat_status scratch_setup(qpat_ctx* c) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (c->device < 0 || c->device >= kMaxDevices)
        return fail(c, QPAT_ERR_DEVICE, "scratch: device %d beyond the %d supported", c->device, kMaxDevices);
    if (g_scratch_ptr[c->device]) return QPAT_OK;
    void* p = nullptr;
    QPAT_HIP(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[c->device] = static_cast<double*>(p);
    return QPAT_OK;
}

qpat_status misfit_noalloc_core(qpat_ctx* c, const double* chi, const double* w, double* out_dev) {
    double* part = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (c->device >= 0 && c->device < kMaxDevices) part = g_scratch_ptr[c->device];
    }
    if (!part) return fail(c, QPAT_ERR_STATE, "misfit_noalloc: no scratch address for device %d", c->device);
    const int64_t n = c->N * c->n_ill;
    const int nb = grid_for(n, kThreads * 8, kRedBlocks);
    if (nb > kRedBlocks)
        return fail(c, QPAT_ERR_ARG, "misfit_noalloc: %d partial sums exceed the scratch of %d", nb, kRedBlocks);
    // every partial the sum reads is written by k_misfit first: nothing to clear
    hipLaunchKernelGGL(k_misfit, dim3(nb), dim3(kThreads), 0, c->stream, c->N, c->n_ill, c->n_pad, chi, w, c->mu,
                       c->phi, part);
    hipLaunchKernelGGL(k_sum_sqrt, dim3(1), dim3(kThreads), 0, c->stream, part, nb, out_dev);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status misfit_core(qpat_ctx* c, const double* chi, const double* w, double* out) {
    const int64_t n = c->N * c->n_ill;
    const int nb = grid_for(n, kThreads * 8, kRedBlocks);
    hipLaunchKernelGGL(k_misfit, dim3(nb), dim3(kThreads), 0, c->stream, c->N, c->n_ill, c->n_pad, chi, w, c->mu,
                       c->phi, c->red_partials);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kThreads), 0, c->stream, c->red_partials, nb, c->red_out);
    QPAT_HIP(c, hipMemcpyAsync(c->red_host, c->red_out, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    *out = std::sqrt(c->red_host[0]);
    return QPAT_OK;
}

qpat_status init_guess_core(qpat_ctx* c, const double* chi, double mu0, double* beta_out) {
    hipLaunchKernelGGL(k_init_guess, dim3(grid_for(c->N, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream, c->N,
                       c->n_ill, c->n_pad, chi, c->phi, mu0, beta_out);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status prior_apply_core(qpat_ctx* c, const double* x, double* y) {
    return spmv64(c, Op::Prior, 1, x, y, 0.0);
}

qpat_status prior_solve_core(qpat_ctx* c, const double* p, double* r, SolveStats* st) {
    const int64_t n2 = 2 * c->N;
    hipLaunchKernelGGL(k_copy, grid1(n2), dim3(kThreads), 0, c->stream, n2, p, c->b64);
    if (mg_ready(c, Op::Prior))
        QPAT_TRY(mg_solve(c, Op::Prior, 1, st));
    else
        QPAT_TRY(pcg_solve(c, Op::Prior, 1, st));
    hipLaunchKernelGGL(k_prior_out, dim3(grid_for(c->N, kThreads, 4096), 2), dim3(kThreads), 0, c->stream, c->N,
                       c->x64, c->scal, r);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// Gram-Schmidt of y (length n) against nb stored vectors; projection coefficients
// are computed against A_j and subtracted along B_j (A = B for the u basis).
static qpat_status reorth(qpat_ctx* c, double* y, int64_t n, const double* A, const double* Bm, int64_t ld, int nb) {
    if (nb <= 0) return QPAT_OK;
    for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < nb; ++j) QPAT_TRY(dot(c, A + j * ld, y, n, c->coef + j));
        hipLaunchKernelGGL(k_sub_combo, grid1(n), dim3(kThreads), 0, c->stream, n, nb, c->coef, Bm, ld, y, c->ls);
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status lsqr_init_core(qpat_ctx* c, const double* chi, const double* w, const double* beta_lin) {
    const int64_t nd = c->N * c->n_pad, n2 = 2 * c->N;
    SolveStats st;
    const double* Jb = nullptr;
    if (beta_lin) {
        const double* bl = beta_lin;
        if (c->ls_kappa_only) {   // J [kt; 0]: c->lr is free until the first M_delta solve
            hipLaunchKernelGGL(k_copy, grid1(c->N), dim3(kThreads), 0, c->stream, c->N, beta_lin, c->lr);
            QPAT_TRY(zero_fill(c, c->lr + c->N, c->N));
            bl = c->lr;
        }
        QPAT_TRY(jvp_core(c, bl, 2, c->dvec, &st));
        Jb = c->dvec;
    }
    hipLaunchKernelGGL(k_lsqr_rhs, dim3(grid_for(nd, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream, c->N,
                       c->n_ill, c->n_pad, chi, w, c->mu, c->phi, Jb, c->lq, c->lw);
    QPAT_TRY(dot(c, c->lq, c->lq, nd, c->red_out));
    hipLaunchKernelGGL(k_ls_init_beta, dim3(1), dim3(64), 0, c->stream, c->ls, c->red_out);
    hipLaunchKernelGGL(k_ls_scale_u, grid1(nd), dim3(kThreads), 0, c->stream, c->ls, nd, c->lq, c->lu, 1);
    QPAT_TRY(vjp_core(c, nullptr, 1, c->lp, &st));
    if (c->ls_kappa_only) QPAT_TRY(zero_fill(c, c->lp + c->N, c->N));
    QPAT_TRY(prior_solve_core(c, c->lp, c->lr, &st));
    QPAT_TRY(dot(c, c->lp, c->lr, n2, c->red_out));
    hipLaunchKernelGGL(k_ls_init_alpha, dim3(1), dim3(64), 0, c->stream, c->ls, c->red_out);
    hipLaunchKernelGGL(k_ls_first_v, grid1(n2), dim3(kThreads), 0, c->stream, c->ls, n2, c->lr, c->lp, c->lv, c->lwh,
                       c->lwd, c->lx);
    c->nbasis = 0;
    c->reorth_on = c->opts.lsqr_reorth != 0;
    if (c->reorth_on) {
        hipLaunchKernelGGL(k_copy, grid1(nd), dim3(kThreads), 0, c->stream, nd, c->lu, c->U);
        hipLaunchKernelGGL(k_copy, grid1(n2), dim3(kThreads), 0, c->stream, n2, c->lv, c->V);
        hipLaunchKernelGGL(k_copy, grid1(n2), dim3(kThreads), 0, c->stream, n2, c->lwh, c->WH);
        c->nbasis = 1;
    }
    QPAT_HIP(c, hipGetLastError());
    QPAT_HIP(c, hipMemcpyAsync(c->ls_host, c->ls, sizeof(LsqrScal), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    if (c->ls_host->breakdown) return fail(c, QPAT_ERR_BREAKDOWN, "LSQR breakdown at initialisation");
    return QPAT_OK;
}

// The stored bases are full: double their capacity (the stored vectors are
// copied over). When the device cannot hold the larger bases the run goes on
// with the plain recurrences (reorthogonalisation off until the next init;
// qpat_lsqr_basis reports 0 then).
static qpat_status grow_bases(qpat_ctx* c) {
    const int64_t nd = c->N * c->n_pad, n2 = 2 * c->N;
    const int cap = 2 * c->basis_cap;
    void *u = nullptr, *v = nullptr, *wh = nullptr, *cf = nullptr;
    bool ok = hipMalloc(&u, (size_t)cap * nd * sizeof(double)) == hipSuccess &&
              hipMalloc(&v, (size_t)cap * n2 * sizeof(double)) == hipSuccess &&
              hipMalloc(&wh, (size_t)cap * n2 * sizeof(double)) == hipSuccess &&
              hipMalloc(&cf, (size_t)cap * sizeof(double)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();   // the failed allocation is not an error of the run
        for (void* p : {u, v, wh, cf})
            if (p) (void)hipFree(p);
        c->reorth_on = false;
        c->nbasis = 0;
        return QPAT_OK;
    }
    const size_t nb = static_cast<size_t>(c->nbasis);
    QPAT_HIP(c, hipMemcpyAsync(u, c->U, nb * nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    QPAT_HIP(c, hipMemcpyAsync(v, c->V, nb * n2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    QPAT_HIP(c, hipMemcpyAsync(wh, c->WH, nb * n2 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    for (double* p : {c->U, c->V, c->WH, c->coef}) QPAT_TRY(dfree(c, p));
    for (void* p : {u, v, wh, cf}) c->allocs.push_back(p);
    c->U = static_cast<double*>(u);
    c->V = static_cast<double*>(v);
    c->WH = static_cast<double*>(wh);
    c->coef = static_cast<double*>(cf);
    c->basis_cap = cap;
    return QPAT_OK;
}

qpat_status lsqr_step_core(qpat_ctx* c, SolveStats* st) {
    const int64_t nd = c->N * c->n_pad, n2 = 2 * c->N;
    if (c->ls_host->done) return QPAT_OK;
    if (c->reorth_on && c->nbasis >= c->basis_cap) QPAT_TRY(grow_bases(c));
    const bool ro = c->reorth_on;
    // q = W J v - alpha u
    QPAT_TRY(jvp_core(c, c->lv, 1, c->lq, st));
    if (ro) QPAT_TRY(reorth(c, c->lq, nd, c->U, c->U, nd, c->nbasis));
    QPAT_TRY(dot(c, c->lq, c->lq, nd, c->red_out));
    hipLaunchKernelGGL(k_ls_beta, dim3(1), dim3(64), 0, c->stream, c->ls, c->red_out);
    hipLaunchKernelGGL(k_ls_lucky, grid1(n2), dim3(kThreads), 0, c->stream, c->ls, n2, c->lx, c->lwd);
    hipLaunchKernelGGL(k_ls_lucky_flag, dim3(1), dim3(64), 0, c->stream, c->ls);
    hipLaunchKernelGGL(k_ls_scale_u, grid1(nd), dim3(kThreads), 0, c->stream, c->ls, nd, c->lq, c->lu, 0);
    // p = W^T... : p = J^T (W u) - beta what
    QPAT_TRY(vjp_core(c, nullptr, 2, c->lp, st));
    if (c->ls_kappa_only) QPAT_TRY(zero_fill(c, c->lp + c->N, c->N));
    if (ro) QPAT_TRY(reorth(c, c->lp, n2, c->V, c->WH, n2, c->nbasis));
    QPAT_TRY(prior_solve_core(c, c->lp, c->lr, st));
    QPAT_TRY(dot(c, c->lp, c->lr, n2, c->red_out));
    hipLaunchKernelGGL(k_ls_rotate, dim3(1), dim3(64), 0, c->stream, c->ls, c->red_out);
    hipLaunchKernelGGL(k_ls_update, grid1(n2), dim3(kThreads), 0, c->stream, c->ls, n2, c->lr, c->lp, c->lv, c->lwh,
                       c->lwd, c->lx);
    hipLaunchKernelGGL(k_ls_alpha_zero, dim3(1), dim3(64), 0, c->stream, c->ls);
    if (ro) {
        hipLaunchKernelGGL(k_copy, grid1(nd), dim3(kThreads), 0, c->stream, nd, c->lu, c->U + c->nbasis * nd);
        hipLaunchKernelGGL(k_copy, grid1(n2), dim3(kThreads), 0, c->stream, n2, c->lv, c->V + c->nbasis * n2);
        hipLaunchKernelGGL(k_copy, grid1(n2), dim3(kThreads), 0, c->stream, n2, c->lwh, c->WH + c->nbasis * n2);
        c->nbasis += 1;
    }
    QPAT_HIP(c, hipGetLastError());
    QPAT_HIP(c, hipMemcpyAsync(c->ls_host, c->ls, sizeof(LsqrScal), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    if (c->ls_host->breakdown) return fail(c, QPAT_ERR_BREAKDOWN, "LSQR breakdown: p.r <= 0 or non-finite");
    return QPAT_OK;
}

}  // namespace qpat
