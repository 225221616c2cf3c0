// Assembly of the P1 system matrix K(kappa, mu), the prior matrix M_delta and
// the load vectors, row by row on the sliced-ELL pattern.
//
// Weak form (Appendix): int kappa grad(phi).grad(v) + mu phi v dx
//   + 1/2 int_bdry phi v dS = 2 int_bdry Phi v dS, kappa and mu P1 interpolants.
// Closed element formulas used here (exact for P1 coefficients):
//   stiffness  S_ab = kbar_T |T| grad(l_a).grad(l_b),   kbar_T = mean of kappa at the 4 vertices
//   mass       M_ab = |T| (1 + d_ab) (s_T + mu_a + mu_b) / 120,   s_T = sum of mu at the vertices
//   boundary   B_ab = |F| (1 + d_ab) / 12
//   load       f_a  = 2 |F| / 12 sum_b (1 + d_ab) Phi_b
// Each thread owns one row and walks the elements around its node in sorted
// order, so the sums are deterministic and need no atomics.
#include "qpat_internal.h"

namespace qpat {
namespace {

struct Grad4 {
    double vol;
    double g[4][3];
};

__device__ __forceinline__ void load_geo(const double* __restrict__ geo, int32_t e, Grad4& G) {
    const double* p = geo + (int64_t)kTetGeo * e;
    G.vol = p[0];
    for (int d = 0; d < 3; ++d) {
        G.g[1][d] = p[1 + d];
        G.g[2][d] = p[4 + d];
        G.g[3][d] = p[7 + d];
        G.g[0][d] = -(G.g[1][d] + G.g[2][d] + G.g[3][d]);
    }
}

__device__ __forceinline__ double dot3(const double* a, const double* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// position of column j in row i (sorted, strided by the slice width)
__device__ __forceinline__ int find_col(const int32_t* __restrict__ cols, int32_t base, int32_t n, int32_t j) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (cols[base + mid * kSlice] < j) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__global__ void k_assemble_K(const Sell s, const int32_t* __restrict__ tets, const double* __restrict__ geo,
                             const int32_t* __restrict__ n2t_ptr, const int32_t* __restrict__ n2t,
                             const int32_t* __restrict__ bf, const double* __restrict__ barea,
                             const int32_t* __restrict__ n2f_ptr, const int32_t* __restrict__ n2f,
                             const double* __restrict__ kappa, const double* __restrict__ mu,
                             double* __restrict__ K64, float* __restrict__ K32, double* __restrict__ dinv64,
                             float* __restrict__ dinv32) {
    int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= s.N) return;
    const int32_t sl = static_cast<int32_t>(row / kSlice);
    const int32_t base = s.slice_ptr[sl] + static_cast<int32_t>(row % kSlice);
    const int32_t w = s.slice_w[sl];
    const int32_t n = s.rowlen[row];
    for (int k = 0; k < w; ++k) K64[base + k * kSlice] = 0.0;
    for (int32_t q = n2t_ptr[row]; q < n2t_ptr[row + 1]; ++q) {
        const int32_t e = n2t[q] >> 2, a = n2t[q] & 3;
        Grad4 G;
        load_geo(geo, e, G);
        int32_t v[4];
        double kb = 0.0, sm = 0.0, m[4];
        for (int b = 0; b < 4; ++b) {
            v[b] = tets[4 * e + b];
            kb += kappa[v[b]];
            m[b] = mu[v[b]];
            sm += m[b];
        }
        kb *= 0.25;
        double ga[3] = {0.0, 0.0, 0.0}, ma = 0.0;   // row vertex a: selected with compile-time indices
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
            for (int d = 0; d < 3; ++d) ga[d] = c == a ? G.g[c][d] : ga[d];
            ma = c == a ? m[c] : ma;
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double val = kb * G.vol * dot3(ga, G.g[b]) +
                         G.vol * (a == b ? 2.0 : 1.0) * (sm + ma + m[b]) * (1.0 / 120.0);
            int pos = find_col(s.cols, base, n, v[b]);
            K64[base + pos * kSlice] += val;
        }
    }
    for (int32_t q = n2f_ptr[row]; q < n2f_ptr[row + 1]; ++q) {
        const int32_t f = n2f[q] / 3, a = n2f[q] % 3;
        const double ar = barea[f];
        for (int b = 0; b < 3; ++b) {
            double val = 0.5 * ar * (a == b ? 2.0 : 1.0) * (1.0 / 12.0);
            int pos = find_col(s.cols, base, n, bf[3 * f + b]);
            K64[base + pos * kSlice] += val;
        }
    }
    for (int k = 0; k < w; ++k) K32[base + k * kSlice] = static_cast<float>(K64[base + k * kSlice]);
    double d = K64[base + s.diag[row] * kSlice];
    dinv64[row] = 1.0 / d;
    dinv32[row] = static_cast<float>(1.0 / d);
}

// Lagged diffusivity c_T = r'(t)/t, t = |grad u_T|, constant per tetrahedron:
//   Perona-Malik (kind 0)  r(t) = (T^2/2) log(1 + t^2/T^2)      c_T = 1 / (1 + t^2/T^2)
//   TV^q (kind 1)          r(t) = T^(2-q) (t^2 + T^2)^(q/2) / q  c_T = (1 + t^2/T^2)^((q-2)/2)
// (qexp = (q - 2) / 2; q = 1 is smoothed total variation).
// blockIdx.y selects the block of M_delta: 0 -> M(kt), 1 -> (b/a) M(mt).
__global__ void k_assemble_prior(const Sell s, const int32_t* __restrict__ tets, const double* __restrict__ geo,
                                 const int32_t* __restrict__ n2t_ptr, const int32_t* __restrict__ n2t,
                                 const double* __restrict__ kt, const double* __restrict__ mt, double invT2,
                                 int kind, double qexp, double b_over_a, double delta, double* __restrict__ M64, float* __restrict__ M32,
                                 double* __restrict__ dinv64, float* __restrict__ dinv32) {
    int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (row >= s.N) return;
    const int sys = blockIdx.y;
    const double* u = sys == 0 ? kt : mt;
    const double scale = sys == 0 ? 1.0 : b_over_a;
    double* V = M64 + sys * s.len;
    float* V32 = M32 + sys * s.len;
    const int32_t sl = static_cast<int32_t>(row / kSlice);
    const int32_t base = s.slice_ptr[sl] + static_cast<int32_t>(row % kSlice);
    const int32_t w = s.slice_w[sl];
    const int32_t n = s.rowlen[row];
    for (int k = 0; k < w; ++k) V[base + k * kSlice] = 0.0;
    for (int32_t q = n2t_ptr[row]; q < n2t_ptr[row + 1]; ++q) {
        const int32_t e = n2t[q] >> 2, a = n2t[q] & 3;
        Grad4 G;
        load_geo(geo, e, G);
        int32_t v[4];
        double gu[3] = {0.0, 0.0, 0.0};
        for (int b = 0; b < 4; ++b) {
            v[b] = tets[4 * e + b];
            double ub = u[v[b]];
            gu[0] += ub * G.g[b][0];
            gu[1] += ub * G.g[b][1];
            gu[2] += ub * G.g[b][2];
        }
        const double s1 = 1.0 + dot3(gu, gu) * invT2;
        const double cT = kind == 0 ? 1.0 / s1 : pow(s1, qexp);
        double ga[3] = {0.0, 0.0, 0.0};   // row vertex a: selected with compile-time indices
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) ga[d] = c == a ? G.g[c][d] : ga[d];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            double val = scale * cT * G.vol * dot3(ga, G.g[b]);
            int pos = find_col(s.cols, base, n, v[b]);
            V[base + pos * kSlice] += val;
        }
    }
    V[base + s.diag[row] * kSlice] += delta;
    for (int k = 0; k < w; ++k) V32[base + k * kSlice] = static_cast<float>(V[base + k * kSlice]);
    double d = V[base + s.diag[row] * kSlice];
    dinv64[sys * s.N + row] = 1.0 / d;
    dinv32[sys * s.N + row] = static_cast<float>(1.0 / d);
}

// f[i][k] = sum over boundary triangles at node i of 2 |F| / 12 sum_b (1 + d_ab) Phi_k,b
__global__ void k_load(int64_t N, int32_t n_ill, int32_t n_pad, int64_t Fb, const double* __restrict__ barea,
                       const int32_t* __restrict__ n2f_ptr, const int32_t* __restrict__ n2f,
                       const double* __restrict__ src, double* __restrict__ f) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * n_pad) return;
    const int64_t row = t / n_pad;
    const int k = static_cast<int>(t % n_pad);
    double acc = 0.0;
    if (k < n_ill) {
        for (int32_t q = n2f_ptr[row]; q < n2f_ptr[row + 1]; ++q) {
            const int32_t fc = n2f[q] / 3, a = n2f[q] % 3;
            const double* P = src + ((int64_t)k * Fb + fc) * 3;
            double sum = P[0] + P[1] + P[2] + P[a];
            acc += 2.0 * barea[fc] * (1.0 / 12.0) * sum;
        }
    }
    f[t] = acc;
}

__global__ void k_exp(int64_t N, double k0, double m0, const double* __restrict__ beta, double* __restrict__ kappa,
                      double* __restrict__ mu) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    kappa[i] = k0 * exp(beta[i]);
    mu[i] = m0 * exp(beta[N + i]);
}

__global__ void k_check_pos(const double* __restrict__ a, int64_t n, int32_t* flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double v = a[i];
        if (!(v > 0.0) || !(v < INFINITY)) atomicOr(flag, 16);
    }
}

}  // namespace

qpat_status assemble_K(qpat_ctx* c) {
    hipLaunchKernelGGL(k_assemble_K, dim3(grid_for(c->N, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream, c->sell,
                       c->tets, c->geo, c->n2t_ptr, c->n2t, c->bfaces, c->barea, c->n2f_ptr, c->n2f, c->kappa, c->mu,
                       c->K64, c->K32, c->Kdinv64, c->Kdinv32);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status assemble_prior(qpat_ctx* c, const double* kt, const double* mt, int kind, double T, double q,
                           double b_over_a, double delta) {
    hipLaunchKernelGGL(k_assemble_prior, dim3(grid_for(c->N, kThreads, 1 << 30), 2), dim3(kThreads), 0, c->stream,
                       c->sell, c->tets, c->geo, c->n2t_ptr, c->n2t, kt, mt, 1.0 / (T * T), kind, 0.5 * (q - 2.0),
                       b_over_a, delta, c->M64,
                       c->M32, c->Mdinv64, c->Mdinv32);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status assemble_load(qpat_ctx* c, const double* phi_src) {
    int64_t items = c->N * c->n_pad;
    hipLaunchKernelGGL(k_load, dim3(grid_for(items, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream, c->N, c->n_ill,
                       c->n_pad, c->Fb, c->barea, c->n2f_ptr, c->n2f, phi_src, c->f);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status exp_params(qpat_ctx* c, double kappa0, double mu0, const double* beta) {
    hipLaunchKernelGGL(k_exp, dim3(grid_for(c->N, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream, c->N, kappa0,
                       mu0, beta, c->kappa, c->mu);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status check_positive(qpat_ctx* c, const double* a, int64_t n, bool* ok) {
    QPAT_HIP(c, hipMemsetAsync(c->dev_flag, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_check_pos, dim3(grid_for(n, kThreads, 8192)), dim3(kThreads), 0, c->stream, a, n,
                       c->dev_flag);
    int32_t flag = 0;
    QPAT_HIP(c, hipMemcpyAsync(&flag, c->dev_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    *ok = flag == 0;
    return QPAT_OK;
}

}  // namespace qpat
