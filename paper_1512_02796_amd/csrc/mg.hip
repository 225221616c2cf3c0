// Geometric multigrid preconditioner for the M_delta solves on lattice meshes.
//
// Each block of M_delta (Sec. 4 eqs. (4.5), (4.8)) is an SPD FEM matrix on the
// node lattice. The solve is PCG preconditioned by one symmetric V-cycle:
//   * levels: the lattice and its vertex-centred coarsenings, n -> n/2 + 1 per
//     axis, down to at most kMgCoarse nodes per axis;
//   * prolongation P: trilinear interpolation (weights 1, 1/2 per axis),
//     restriction P^T;
//   * coarse operators by Galerkin products A_c = P^T A P, stored like the fine
//     stencil form (diagonal + upper offsets, node-major), 27-point;
//   * smoother: kMgNu Jacobi sweeps before and after the coarse correction,
//     weight 4/(3 g) with g >= lambda_max(D^{-1} A) the Gershgorin bound;
//   * coarsest level: the explicit inverse (dense, computed on the host).
// With deflation (the exact eigenpair (delta, 1) of each block) the solve runs
// on the complement of the constants as the Jacobi-PCG path does: b <- b -
// mean(b), z <- V(r) - mean(V(r)), and the mean of the solution is mean(b)/delta.
// The stopping rule is the same: ||b - A x||_2 <= rtol ||b||_2 on the FP64
// residual, confirmed on the true residual at the end.
#include <cmath>
#include <cstring>

#include "qpat_internal.h"

namespace qpat {

struct MgLevel {
    int32_t nx = 0, ny = 0, nz = 0;
    int64_t N = 0;
    int32_t m = 0;                 // stored upper offsets
    int32_t kind = 0;              // row kernel: 0 generic table, 1 Kuhn offsets, 2 full 27-point
    const int4* tab = nullptr;     // [m]: dx, dy, dz, dx + nx (dy + ny dz)
    int4* tab_own = nullptr;
    double* U = nullptr;           // [2][N][m+1] (level 0: the context's MU64)
    double* dinv = nullptr;        // [2][N] 1 / a_ii
    double* b = nullptr;           // [2][N] (level 0: the PCG residual)
    double* x = nullptr;           // [2][N]
    double* t = nullptr;           // [2][N] ping-pong partner of x
    double* r = nullptr;           // [2][N] residual before restriction
};

struct MgScal {
    double rz, pq, alpha, beta, c, rr, bnorm2, mean;
    int32_t active, done, iters, pad;
};

struct MgState {
    std::vector<MgLevel> lv;
    double* w = nullptr;           // [2][levels] Jacobi weights
    double* ainv = nullptr;        // [2][Nc][Nc]
    double *pr = nullptr, *pp = nullptr, *pq = nullptr;  // PCG r, p, q: [2][N]
    double* parts = nullptr;       // [2][4][kMgBlocks]
    uint64_t* gmax = nullptr;      // [2][levels] Gershgorin bounds (bit patterns)
    MgScal* sc = nullptr;          // [2]
    MgScal* sc_host = nullptr;
    double* zout = nullptr;        // where the V-cycle leaves z
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap = nullptr;
};

namespace {

constexpr int kMgCoarse = 5;      // coarsest lattice: at most this many nodes per axis
constexpr int kMgNu = 1;          // Jacobi sweeps before and after the coarse correction
constexpr int kMgBlocks = 512;    // blocks per system of the vector kernels (partial sums)
constexpr int kMgT = 256;

__device__ __forceinline__ void coords(int32_t i, int nx, int ny, int& ix, int& iy, int& iz) {
    ix = i % nx;
    const int32_t q = i / nx;
    iy = q % ny;
    iz = q / ny;
}

// (A x)_i, and sum_j |a_ij| when ABS
template <bool ABS>
__device__ __forceinline__ double st_row(const double* __restrict__ U, int M1, const int4* __restrict__ tab, int m,
                                         int nx, int ny, int nz, const double* __restrict__ x, int32_t i) {
    int ix, iy, iz;
    coords(i, nx, ny, ix, iy, iz);
    double s = ABS ? fabs(U[(int64_t)i * M1]) : U[(int64_t)i * M1] * x[i];
    for (int j = 0; j < m; ++j) {
        const int4 t = tab[j];
        const int ux = ix + t.x, uy = iy + t.y, uz = iz + t.z;
        if (ux >= 0 && ux < nx && uy >= 0 && uy < ny && uz < nz) {
            const double a = U[(int64_t)i * M1 + j + 1];
            s += ABS ? fabs(a) : a * x[i + t.w];
        }
        const int lx = ix - t.x, ly = iy - t.y, lz = iz - t.z;
        if (lx >= 0 && lx < nx && ly >= 0 && ly < ny && lz >= 0) {
            const double a = U[(int64_t)(i - t.w) * M1 + j + 1];
            s += ABS ? fabs(a) : a * x[i - t.w];
        }
    }
    return s;
}

// The same row with compile-time offsets: KIND 1 the Kuhn split (7 upper
// offsets, the fine level), KIND 2 the full 27-point stencil (13 upper offsets
// in code order, the Galerkin levels); KIND 0 the generic table. Interior rows
// skip the lattice-edge tests.
constexpr int kKx[7] = {1, 0, 1, 0, 1, 0, 1};
constexpr int kKy[7] = {0, 1, 1, 0, 0, 1, 1};
constexpr int kKz[7] = {0, 0, 0, 1, 1, 1, 1};

template <int KIND>
__device__ __forceinline__ double st_apply(const double* __restrict__ U, int M1, const int4* __restrict__ tab, int m,
                                           int nx, int ny, int nz, const double* __restrict__ x, int32_t i) {
    if constexpr (KIND == 0) {
        return st_row<false>(U, M1, tab, m, nx, ny, nz, x, i);
    } else {
        constexpr int MM = KIND == 1 ? 7 : 13;
        int ix, iy, iz;
        coords(i, nx, ny, ix, iy, iz);
        const bool inner = ix > 0 && ix < nx - 1 && iy > 0 && iy < ny - 1 && iz > 0 && iz < nz - 1;
        const double* __restrict__ Ui = U + (int64_t)i * (MM + 1);
        double s = Ui[0] * x[i];
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            const int code = 14 + j;
            const int dx = KIND == 1 ? kKx[j] : code % 3 - 1;
            const int dy = KIND == 1 ? kKy[j] : (code / 3) % 3 - 1;
            const int dz = KIND == 1 ? kKz[j] : code / 9 - 1;
            const int32_t lin = dx + nx * (dy + ny * dz);
            const bool up = inner || (ix + dx >= 0 && ix + dx < nx && iy + dy >= 0 && iy + dy < ny && iz + dz < nz);
            const bool lo = inner || (ix - dx >= 0 && ix - dx < nx && iy - dy >= 0 && iy - dy < ny && iz - dz >= 0);
            if (up) s += Ui[j + 1] * x[i + lin];
            if (lo) s += U[(int64_t)(i - lin) * (MM + 1) + j + 1] * x[i - lin];
        }
        return s;
    }
}

// XCD-aware row loop for the stencil kernels: block b runs on XCD b mod 8,
// so each XCD takes a contiguous eighth of the rows and its blocks sweep it
// together; the partner rows one plane back are then still in that XCD's L2.
#define QPAT_MG_ROWS(i, N)                                                                      \
    const int32_t _per = gridDim.x >> 3;                                                       \
    const int64_t _chunk = ((N) + 7) / 8;                                                      \
    const int64_t _lo = (blockIdx.x & 7) * _chunk;                                             \
    const int64_t _hi = _lo + _chunk < (N) ? _lo + _chunk : (N);                               \
    for (int64_t i = _lo + (int64_t)(blockIdx.x >> 3) * kMgT + threadIdx.x; i < _hi; i += (int64_t)_per * kMgT)

__device__ __forceinline__ double bsum(double v, double* sm) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kMgT / 64; ++w) t += sm[w];
    __syncthreads();
    return t;
}

struct LvArgs {
    const double* U;
    const int4* tab;
    int32_t m, nx, ny, nz;
    int64_t N;
    int32_t kind;         // 0 generic table, 1 Kuhn offsets, 2 full 27-point
};

// 1 / a_ii and the Gershgorin bound max_i sum_j |a_ij| / a_ii
__global__ __launch_bounds__(kMgT) void k_mg_diag(LvArgs L, double* __restrict__ dinv, uint64_t* __restrict__ gmax,
                                                  int nlev, int lev) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    const int M1 = L.m + 1;
    const double* U = L.U + (int64_t)sys * L.N * M1;
    double g = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        const double d = U[i * M1];
        dinv[sys * L.N + i] = 1.0 / d;
        const double row = st_row<true>(U, M1, L.tab, L.m, L.nx, L.ny, L.nz, nullptr, static_cast<int32_t>(i));
        g = fmax(g, row / d);
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) g = fmax(g, __shfl_xor(g, off));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = g;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kMgT / 64; ++w) t = fmax(t, sm[w]);
        // positive doubles order like their bit patterns
        atomicMax(reinterpret_cast<unsigned long long*>(gmax + sys * nlev + lev),
                  static_cast<unsigned long long>(__double_as_longlong(t)));
    }
}

__device__ __forceinline__ double pw(int d) { return d == 0 ? 1.0 : 0.5; }

// Galerkin coarse operator A_c = P^T A P, diagonal and the 13 upper offsets
// (code order (dx+1) + 3 (dy+1) + 9 (dz+1) = 13 ... 26) of every coarse node:
// sum over the fine nodes i in the support of I, the fine stencil entries
// a_ij, and the coarse nodes J whose support holds j, of P(i,I) a_ij P(j,J).
__global__ __launch_bounds__(kMgT) void k_mg_rap(LvArgs F, double* __restrict__ Uc, int cx, int cy, int cz) {
    __shared__ double acc[kMgT][14];
    const int sys = blockIdx.y;
    const int64_t Nc = (int64_t)cx * cy * cz;
    const int64_t I = blockIdx.x * (int64_t)kMgT + threadIdx.x;
    const int Mf = F.m + 1;
    const double* U = F.U + (int64_t)sys * F.N * Mf;
    for (int k = 0; k < 14; ++k) acc[threadIdx.x][k] = 0.0;
    if (I < Nc) {
        int Ix, Iy, Iz;
        coords(static_cast<int32_t>(I), cx, cy, Ix, Iy, Iz);
        for (int di = 0; di < 27; ++di) {
            const int ax = di % 3 - 1, ay = (di / 3) % 3 - 1, az = di / 9 - 1;
            const int fx = 2 * Ix + ax, fy = 2 * Iy + ay, fz = 2 * Iz + az;
            if (fx < 0 || fx >= F.nx || fy < 0 || fy >= F.ny || fz < 0 || fz >= F.nz) continue;
            const double wi = pw(ax) * pw(ay) * pw(az);
            const int32_t i = fx + F.nx * (fy + F.ny * fz);
            // the fine row: diagonal, upper and lower entries
            for (int s = -F.m; s <= F.m; ++s) {
                int sx = 0, sy = 0, sz = 0, lin = 0;
                double a;
                if (s == 0) {
                    a = U[(int64_t)i * Mf];
                } else {
                    const int4 t = F.tab[(s > 0 ? s : -s) - 1];
                    const int sg = s > 0 ? 1 : -1;
                    sx = sg * t.x;
                    sy = sg * t.y;
                    sz = sg * t.z;
                    lin = sg * t.w;
                    const int jx = fx + sx, jy = fy + sy, jz = fz + sz;
                    if (jx < 0 || jx >= F.nx || jy < 0 || jy >= F.ny || jz < 0 || jz >= F.nz) continue;
                    a = s > 0 ? U[(int64_t)i * Mf + s] : U[(int64_t)(i + lin) * Mf + (-s)];
                }
                const int jx = fx + sx, jy = fy + sy, jz = fz + sz;
                // coarse nodes J with j in their support: per axis one (even) or two (odd)
                const int x0 = jx >> 1, x1 = (jx + 1) >> 1;
                const int y0 = jy >> 1, y1 = (jy + 1) >> 1;
                const int z0 = jz >> 1, z1 = (jz + 1) >> 1;
                for (int Jz = z0; Jz <= z1; ++Jz) {
                    if (Jz >= cz) continue;
                    const double wz = pw(jz - 2 * Jz);
                    for (int Jy = y0; Jy <= y1; ++Jy) {
                        if (Jy >= cy) continue;
                        const double wy = pw(jy - 2 * Jy);
                        for (int Jx = x0; Jx <= x1; ++Jx) {
                            if (Jx >= cx) continue;
                            const int code = (Jx - Ix + 1) + 3 * (Jy - Iy + 1) + 9 * (Jz - Iz + 1);
                            if (code < 13) continue;   // lower half: stored at the partner row
                            acc[threadIdx.x][code - 13] += wi * a * wz * wy * pw(jx - 2 * Jx);
                        }
                    }
                }
            }
        }
        double* out = Uc + ((int64_t)sys * Nc + I) * 14;
        for (int k = 0; k < 14; ++k) out[k] = acc[threadIdx.x][k];
    }
}

struct SmArgs {
    LvArgs L;
    const double* dinv;
    const double* w;     // [2][levels]
    int32_t nlev, lev;
    const MgScal* sc;
};

// x = w D^{-1} b (first sweep from zero)
__global__ __launch_bounds__(kMgT) void k_mg_first(SmArgs a, const double* __restrict__ b, double* __restrict__ x) {
    const int sys = blockIdx.y;
    if (!a.sc[sys].active) return;
    const double w = a.w[sys * a.nlev + a.lev];
    const int64_t o = sys * a.L.N;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT)
        x[o + i] = w * a.dinv[o + i] * b[o + i];
}

// y = x + w D^{-1} (b - A x)
template <int KIND>
// The two systems are swept one after the other by the same blocks (not
// side by side): each XCD's L2 then holds the band of one system only.
__global__ __launch_bounds__(kMgT) void k_mg_smooth(SmArgs a, const double* __restrict__ b,
                                                    const double* __restrict__ x, double* __restrict__ y) {
    for (int sys = 0; sys < 2; ++sys) {
        if (!a.sc[sys].active) continue;
        const double w = a.w[sys * a.nlev + a.lev];
        const int M1 = a.L.m + 1;
        const int64_t o = sys * a.L.N;
        const double* U = a.L.U + o * M1;
        QPAT_MG_ROWS(i, a.L.N) {
            const double ax = st_apply<KIND>(U, M1, a.L.tab, a.L.m, a.L.nx, a.L.ny, a.L.nz, x + o, (int32_t)i);
            y[o + i] = x[o + i] + w * a.dinv[o + i] * (b[o + i] - ax);
        }
    }
}

// r = b - A x
template <int KIND>
__global__ __launch_bounds__(kMgT) void k_mg_resid(SmArgs a, const double* __restrict__ b,
                                                   const double* __restrict__ x, double* __restrict__ r) {
    for (int sys = 0; sys < 2; ++sys) {
        if (!a.sc[sys].active) continue;
        const int M1 = a.L.m + 1;
        const int64_t o = sys * a.L.N;
        const double* U = a.L.U + o * M1;
        QPAT_MG_ROWS(i, a.L.N)
            r[o + i] = b[o + i] - st_apply<KIND>(U, M1, a.L.tab, a.L.m, a.L.nx, a.L.ny, a.L.nz, x + o, (int32_t)i);
    }
}

// bc = P^T r
__global__ __launch_bounds__(kMgT) void k_mg_restrict(int nx, int ny, int nz, int cx, int cy, int cz,
                                                      const double* __restrict__ r, double* __restrict__ bc,
                                                      const MgScal* __restrict__ sc) {
    const int sys = blockIdx.y;
    if (!sc[sys].active) return;
    const int64_t Nf = (int64_t)nx * ny * nz, Nc = (int64_t)cx * cy * cz;
    for (int64_t I = blockIdx.x * (int64_t)kMgT + threadIdx.x; I < Nc; I += (int64_t)gridDim.x * kMgT) {
        int Ix, Iy, Iz;
        coords((int32_t)I, cx, cy, Ix, Iy, Iz);
        double s = 0.0;
        for (int az = -1; az <= 1; ++az) {
            const int fz = 2 * Iz + az;
            if (fz < 0 || fz >= nz) continue;
            for (int ay = -1; ay <= 1; ++ay) {
                const int fy = 2 * Iy + ay;
                if (fy < 0 || fy >= ny) continue;
                for (int ax = -1; ax <= 1; ++ax) {
                    const int fx = 2 * Ix + ax;
                    if (fx < 0 || fx >= nx) continue;
                    s += pw(ax) * pw(ay) * pw(az) * r[sys * Nf + fx + (int64_t)nx * (fy + (int64_t)ny * fz)];
                }
            }
        }
        bc[sys * Nc + I] = s;
    }
}

// x += P xc
__global__ __launch_bounds__(kMgT) void k_mg_prolong(int nx, int ny, int nz, int cx, int cy, int cz,
                                                     const double* __restrict__ xc, double* __restrict__ x,
                                                     const MgScal* __restrict__ sc) {
    const int sys = blockIdx.y;
    if (!sc[sys].active) return;
    const int64_t Nf = (int64_t)nx * ny * nz, Nc = (int64_t)cx * cy * cz;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < Nf; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords((int32_t)i, nx, ny, ix, iy, iz);
        double s = 0.0;
        for (int Jz = iz >> 1; Jz <= (iz + 1) >> 1; ++Jz) {
            if (Jz >= cz) continue;
            for (int Jy = iy >> 1; Jy <= (iy + 1) >> 1; ++Jy) {
                if (Jy >= cy) continue;
                for (int Jx = ix >> 1; Jx <= (ix + 1) >> 1; ++Jx) {
                    if (Jx >= cx) continue;
                    s += pw(ix - 2 * Jx) * pw(iy - 2 * Jy) * pw(iz - 2 * Jz) *
                         xc[sys * Nc + Jx + (int64_t)cx * (Jy + (int64_t)cy * Jz)];
                }
            }
        }
        x[sys * Nf + i] += s;
    }
}

// x = Ainv b on the coarsest level
__global__ __launch_bounds__(kMgT) void k_mg_dense(int64_t Nc, const double* __restrict__ ainv,
                                                   const double* __restrict__ b, double* __restrict__ x,
                                                   const MgScal* __restrict__ sc) {
    const int sys = blockIdx.y;
    if (!sc[sys].active) return;
    const double* A = ainv + sys * Nc * Nc;
    for (int64_t I = blockIdx.x * (int64_t)kMgT + threadIdx.x; I < Nc; I += (int64_t)gridDim.x * kMgT) {
        double s = 0.0;
        for (int64_t J = 0; J < Nc; ++J) s += A[I * Nc + J] * b[sys * Nc + J];
        x[sys * Nc + I] = s;
    }
}

// ---------------------------------------------------------------- PCG kernels
struct PcgMg {
    LvArgs L;             // the fine operator
    double* x;            // [2][N] iterate
    double* r;
    double* p;
    double* q;
    const double* z;
    double* parts;        // [2][4][kMgBlocks]
    MgScal* sc;
    double rtol2;
    int32_t maxit, deflate;
    int32_t nb;           // blocks per system of the vector kernels (partials written)
};

__device__ __forceinline__ void put(double* parts, int sys, int v, double val) {
    parts[(sys * 4 + v) * kMgBlocks + blockIdx.x] = val;
}

// p = z - c + beta p
__global__ __launch_bounds__(kMgT) void k_mgp_dir(PcgMg a) {
    const int sys = blockIdx.y;
    const MgScal s = a.sc[sys];
    if (!s.active) return;
    const int64_t o = sys * a.L.N;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT)
        a.p[o + i] = a.z[o + i] - s.c + s.beta * a.p[o + i];
}

// q = A p, partial p.q
template <int KIND>
__global__ __launch_bounds__(kMgT) void k_mgp_spmv(PcgMg a) {
    __shared__ double sm[kMgT / 64];
    for (int sys = 0; sys < 2; ++sys) {
        if (!a.sc[sys].active) continue;
        const int M1 = a.L.m + 1;
        const int64_t o = sys * a.L.N;
        const double* U = a.L.U + o * M1;
        double pq = 0.0;
        QPAT_MG_ROWS(i, a.L.N) {
            const double v = st_apply<KIND>(U, M1, a.L.tab, a.L.m, a.L.nx, a.L.ny, a.L.nz, a.p + o, (int32_t)i);
            a.q[o + i] = v;
            pq += a.p[o + i] * v;
        }
        pq = bsum(pq, sm);
        if (threadIdx.x == 0) put(a.parts, sys, 0, pq);
    }
}

// x += alpha p, r -= alpha q, partial r.r
__global__ __launch_bounds__(kMgT) void k_mgp_update(PcgMg a) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    const MgScal s = a.sc[sys];
    if (!s.active) return;
    const int64_t o = sys * a.L.N;
    double rr = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT) {
        a.x[o + i] += s.alpha * a.p[o + i];
        const double ri = a.r[o + i] - s.alpha * a.q[o + i];
        a.r[o + i] = ri;
        rr += ri * ri;
    }
    rr = bsum(rr, sm);
    if (threadIdx.x == 0) put(a.parts, sys, 1, rr);
}

// partial r.z, sum z, sum r (after the V-cycle)
__global__ __launch_bounds__(kMgT) void k_mgp_dots(PcgMg a) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    if (!a.sc[sys].active) return;
    const int64_t o = sys * a.L.N;
    double rz = 0.0, z1 = 0.0, r1 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT) {
        rz += a.r[o + i] * a.z[o + i];
        z1 += a.z[o + i];
        r1 += a.r[o + i];
    }
    rz = bsum(rz, sm);
    z1 = bsum(z1, sm);
    r1 = bsum(r1, sm);
    if (threadIdx.x == 0) {
        put(a.parts, sys, 0, rz);
        put(a.parts, sys, 2, z1);
        put(a.parts, sys, 3, r1);
    }
}

__device__ double red(const double* parts, int nb, int sys, int v, double* sm) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += parts[(sys * 4 + v) * kMgBlocks + b];
    return bsum(s, sm);
}

// phase 0: alpha = rz / pq; phase 1: rr, convergence, iteration count;
// phase 2 (after the V-cycle): c, beta, rz; phase 3: start of a run (r = b,
// after its V-cycle): c, rz, beta = 0
__global__ __launch_bounds__(kMgT) void k_mgp_scalars(PcgMg a, int phase) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    if (!a.sc[sys].active) return;
    MgScal& s = a.sc[sys];
    if (phase == 0) {
        const double pq = red(a.parts, a.nb, sys, 0, sm);
        if (threadIdx.x == 0) {
            s.pq = pq;
            s.alpha = pq != 0.0 ? s.rz / pq : 0.0;
        }
    } else if (phase == 1) {
        const double rr = red(a.parts, a.nb, sys, 1, sm);
        if (threadIdx.x == 0) {
            s.rr = rr;
            s.iters += 1;
            if (rr <= a.rtol2 * s.bnorm2) {
                s.done = 1;
                s.active = 0;
            } else if (s.iters >= a.maxit) {
                s.active = 0;
            }
        }
    } else {
        double rz = red(a.parts, a.nb, sys, 0, sm);
        const double z1 = red(a.parts, a.nb, sys, 2, sm);
        const double r1 = red(a.parts, a.nb, sys, 3, sm);
        if (threadIdx.x == 0) {
            const double c = a.deflate ? z1 / static_cast<double>(a.L.N) : 0.0;
            rz -= c * r1;     // r.(z - c)
            s.c = c;
            s.beta = (phase == 2 && s.rz != 0.0) ? rz / s.rz : 0.0;
            s.rz = rz;
        }
    }
}

// b <- b - mean(b) per system (deflation), ||b||^2 of the original b
__global__ __launch_bounds__(kMgT) void k_mgp_bstats(PcgMg a, const double* __restrict__ b) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    const int64_t o = sys * a.L.N;
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT) {
        s1 += b[o + i];
        s2 += b[o + i] * b[o + i];
    }
    s1 = bsum(s1, sm);
    s2 = bsum(s2, sm);
    if (threadIdx.x == 0) {
        put(a.parts, sys, 2, s1);
        put(a.parts, sys, 3, s2);
    }
}

__global__ __launch_bounds__(kMgT) void k_mgp_init(PcgMg a, double inv_delta) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    const double s1 = red(a.parts, a.nb, sys, 2, sm);
    const double s2 = red(a.parts, a.nb, sys, 3, sm);
    if (threadIdx.x == 0) {
        MgScal& s = a.sc[sys];
        const double mean = a.deflate ? s1 / static_cast<double>(a.L.N) : 0.0;
        s.c = mean;                       // subtracted from b by k_mgp_start
        s.mean = mean * inv_delta;
        s.bnorm2 = s2;
        s.rz = s.pq = s.alpha = s.beta = 0.0;
        s.rr = s2;
        s.iters = 0;
        s.done = s2 == 0.0 ? 1 : 0;
        s.active = s2 == 0.0 ? 0 : 1;
    }
}

// r = b - mean, x = 0, p = 0
__global__ __launch_bounds__(kMgT) void k_mgp_start(PcgMg a, double* __restrict__ b) {
    const int sys = blockIdx.y;
    const double m = a.sc[sys].c;
    const int64_t o = sys * a.L.N;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < a.L.N; i += (int64_t)gridDim.x * kMgT) {
        b[o + i] -= m;
        a.r[o + i] = b[o + i];
        a.x[o + i] = 0.0;
        a.p[o + i] = 0.0;
    }
}

// true residual r = b - A x, partial r.r (restart of a run: r replaces the recursive residual)
__global__ __launch_bounds__(kMgT) void k_mgp_true(PcgMg a, const double* __restrict__ b) {
    __shared__ double sm[kMgT / 64];
    for (int sys = 0; sys < 2; ++sys) {
        const int M1 = a.L.m + 1;
        const int64_t o = sys * a.L.N;
        const double* U = a.L.U + o * M1;
        double rr = 0.0;
        QPAT_MG_ROWS(i, a.L.N) {
            const double ri =
                b[o + i] - st_row<false>(U, M1, a.L.tab, a.L.m, a.L.nx, a.L.ny, a.L.nz, a.x + o, (int32_t)i);
            a.r[o + i] = ri;
            rr += ri * ri;
        }
        rr = bsum(rr, sm);
        if (threadIdx.x == 0) put(a.parts, sys, 1, rr);
    }
}

__global__ void k_mgp_true_fin(PcgMg a, int reopen) {
    __shared__ double sm[kMgT / 64];
    const int sys = blockIdx.y;
    const double rr = red(a.parts, a.nb, sys, 1, sm);
    if (threadIdx.x == 0) {
        MgScal& s = a.sc[sys];
        s.rr = rr;
        const bool ok = rr <= a.rtol2 * s.bnorm2;
        s.done = ok ? 1 : 0;
        s.active = (!ok && reopen && s.iters < a.maxit) ? 1 : 0;
        s.rz = 0.0;   // a reopened run restarts its Krylov space from the true residual
    }
}

inline LvArgs lv_args(const MgLevel& L) {
    LvArgs a;
    a.U = L.U;
    a.tab = L.tab;
    a.m = L.m;
    a.nx = L.nx;
    a.ny = L.ny;
    a.nz = L.nz;
    a.N = L.N;
    a.kind = L.kind;
    return a;
}

// a multiple of 8 blocks per system (the XCD row split), at most kMgBlocks
inline dim3 vgrid(int64_t n) { return dim3((grid_for(n, kMgT, kMgBlocks) + 7) & ~7, 2); }
// the stencil kernels loop over the two systems themselves
inline dim3 sgrid(int64_t n) { return dim3(vgrid(n).x, 1); }

#define QPAT_MG_KIND(kind, KERNEL, ...)                                                   \
    switch (kind) {                                                                        \
        case 1: hipLaunchKernelGGL(KERNEL<1>, __VA_ARGS__); break;                         \
        case 2: hipLaunchKernelGGL(KERNEL<2>, __VA_ARGS__); break;                         \
        default: hipLaunchKernelGGL(KERNEL<0>, __VA_ARGS__); break;                        \
    }

// Dense inverse of an SPD matrix (Cholesky), in place; false if not positive definite.
bool spd_inverse(std::vector<double>& A, int n) {
    std::vector<double> L(A);
    for (int j = 0; j < n; ++j) {
        double d = L[(size_t)j * n + j];
        for (int k = 0; k < j; ++k) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) return false;
        d = std::sqrt(d);
        L[(size_t)j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double s = L[(size_t)i * n + j];
            for (int k = 0; k < j; ++k) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / d;
        }
    }
    // columns of the inverse: solve L L^T x = e_c
    std::vector<double> y(n);
    for (int col = 0; col < n; ++col) {
        for (int i = 0; i < n; ++i) {
            double s = i == col ? 1.0 : 0.0;
            for (int k = 0; k < i; ++k) s -= L[(size_t)i * n + k] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = y[i];
            for (int k = i + 1; k < n; ++k) s -= L[(size_t)k * n + i] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int i = 0; i < n; ++i) A[(size_t)i * n + col] = y[i];
    }
    return true;
}

// one V-cycle on both systems: z = V(b_0); returns the buffer that holds z
// (launch = false: only that buffer, nothing enqueued)
double* vcycle(qpat_ctx* c, hipStream_t st, bool launch = true) {
    MgState& M = *c->mg;
    const int nl = static_cast<int>(M.lv.size());
    std::vector<double*> xl(nl), tl(nl);
    for (int l = 0; l < nl; ++l) {
        xl[l] = M.lv[l].x;
        tl[l] = M.lv[l].t;
    }
    auto sm = [&](int l) {
        SmArgs a;
        a.L = lv_args(M.lv[l]);
        a.dinv = M.lv[l].dinv;
        a.w = M.w;
        a.nlev = nl;
        a.lev = l;
        a.sc = M.sc;
        return a;
    };
    // level 0 takes 2 kMgNu - 1 ping-pong sweeps (odd): z ends in t
    if (!launch) return nl > 1 ? tl[0] : xl[0];
    for (int l = 0; l < nl - 1; ++l) {
        const MgLevel& L = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        const SmArgs a = sm(l);
        hipLaunchKernelGGL(k_mg_first, vgrid(L.N), dim3(kMgT), 0, st, a, L.b, xl[l]);
        for (int k = 1; k < kMgNu; ++k) {
            QPAT_MG_KIND(L.kind, k_mg_smooth, sgrid(L.N), dim3(kMgT), 0, st, a, L.b, xl[l], tl[l]);
            std::swap(xl[l], tl[l]);
        }
        QPAT_MG_KIND(L.kind, k_mg_resid, sgrid(L.N), dim3(kMgT), 0, st, a, L.b, xl[l], L.r);
        hipLaunchKernelGGL(k_mg_restrict, vgrid(C.N), dim3(kMgT), 0, st, L.nx, L.ny, L.nz, C.nx, C.ny, C.nz, L.r, C.b,
                           M.sc);
    }
    const MgLevel& K = M.lv[nl - 1];
    hipLaunchKernelGGL(k_mg_dense, vgrid(K.N), dim3(kMgT), 0, st, K.N, M.ainv, K.b, xl[nl - 1], M.sc);
    for (int l = nl - 2; l >= 0; --l) {
        const MgLevel& L = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        const SmArgs a = sm(l);
        hipLaunchKernelGGL(k_mg_prolong, vgrid(L.N), dim3(kMgT), 0, st, L.nx, L.ny, L.nz, C.nx, C.ny, C.nz, xl[l + 1],
                           xl[l], M.sc);
        for (int k = 0; k < kMgNu; ++k) {
            QPAT_MG_KIND(L.kind, k_mg_smooth, sgrid(L.N), dim3(kMgT), 0, st, a, L.b, xl[l], tl[l]);
            std::swap(xl[l], tl[l]);
        }
    }
    return xl[0];
}

PcgMg pcg_args(qpat_ctx* c) {
    MgState& M = *c->mg;
    PcgMg a;
    a.L = lv_args(M.lv[0]);
    a.x = c->x64;
    a.r = M.pr;
    a.p = M.pp;
    a.q = M.pq;
    a.z = M.zout;
    a.parts = M.parts;
    a.sc = M.sc;
    a.rtol2 = c->opts.prior_rtol * c->opts.prior_rtol;
    a.maxit = c->opts.pcg_maxit;
    a.deflate = c->opts.prior_deflate;
    a.nb = static_cast<int32_t>(vgrid(c->N).x);
    return a;
}

// one iteration after the first direction: direction, SpMV, alpha, update,
// rr, V-cycle, dots, beta
void iteration(qpat_ctx* c, const PcgMg& a, hipStream_t st) {
    const dim3 g = vgrid(a.L.N), one(1, 2);
    hipLaunchKernelGGL(k_mgp_dir, g, dim3(kMgT), 0, st, a);
    QPAT_MG_KIND(a.L.kind, k_mgp_spmv, sgrid(a.L.N), dim3(kMgT), 0, st, a);
    hipLaunchKernelGGL(k_mgp_scalars, one, dim3(kMgT), 0, st, a, 0);
    hipLaunchKernelGGL(k_mgp_update, g, dim3(kMgT), 0, st, a);
    hipLaunchKernelGGL(k_mgp_scalars, one, dim3(kMgT), 0, st, a, 1);
    (void)vcycle(c, st);
    hipLaunchKernelGGL(k_mgp_dots, g, dim3(kMgT), 0, st, a);
    hipLaunchKernelGGL(k_mgp_scalars, one, dim3(kMgT), 0, st, a, 2);
}

}  // namespace

void mg_destroy(qpat_ctx* c) {
    if (!c->mg) return;
    for (auto& kv : c->mg->graphs) (void)hipGraphExecDestroy(kv.second);
    if (c->mg->cap) (void)hipStreamDestroy(c->mg->cap);
    if (c->mg->sc_host) (void)hipHostFree(c->mg->sc_host);
    delete c->mg;
    c->mg = nullptr;
}

bool mg_available(const qpat_ctx* c) {
    return c->lat.on && c->opts.operator_format == 1 && c->opts.prior_precond == 1 && c->MU64 &&
           (int64_t)(c->lat.m + 1) * c->N * 8 < (int64_t(1) << 31);
}

// Hierarchy for the current M_delta (after prior assembly and its stencil form).
qpat_status mg_setup(qpat_ctx* c) {
    if (!mg_available(c)) return QPAT_OK;
    if (!c->mg) {
        c->mg = new MgState();
        MgState& M = *c->mg;
        MgLevel L0;
        L0.nx = c->lat.nx;
        L0.ny = c->lat.ny;
        L0.nz = c->lat.nz;
        L0.N = c->N;
        L0.m = c->lat.m;
        L0.tab = reinterpret_cast<const int4*>(c->lat_tab);
        bool kuhn = c->lat.m == 7;
        for (int j = 0; kuhn && j < 7; ++j)
            kuhn = c->lat.dx[j] == kKx[j] && c->lat.dy[j] == kKy[j] && c->lat.dz[j] == kKz[j];
        L0.kind = kuhn ? 1 : 0;
        M.lv.push_back(L0);
        while (std::max(M.lv.back().nx, std::max(M.lv.back().ny, M.lv.back().nz)) > kMgCoarse) {
            const MgLevel& F = M.lv.back();
            MgLevel C;
            C.nx = F.nx > 2 ? F.nx / 2 + 1 : F.nx;
            C.ny = F.ny > 2 ? F.ny / 2 + 1 : F.ny;
            C.nz = F.nz > 2 ? F.nz / 2 + 1 : F.nz;
            if (C.nx == F.nx && C.ny == F.ny && C.nz == F.nz) break;
            C.N = (int64_t)C.nx * C.ny * C.nz;
            C.m = 13;
            C.kind = 2;
            M.lv.push_back(C);
        }
        const int nl = static_cast<int>(M.lv.size());
        const int64_t Nc = M.lv.back().N;
        if (Nc > 4096) {   // dense coarsest solve would be too large: keep Jacobi-PCG
            mg_destroy(c);
            return QPAT_OK;
        }
        for (int l = 0; l < nl; ++l) {
            MgLevel& L = M.lv[l];
            if (l > 0) {
                int32_t tab[4 * 13];
                for (int j = 0; j < 13; ++j) {
                    const int code = 14 + j;
                    const int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
                    tab[4 * j] = dx;
                    tab[4 * j + 1] = dy;
                    tab[4 * j + 2] = dz;
                    tab[4 * j + 3] = dx + L.nx * (dy + L.ny * dz);
                }
                QPAT_TRY(dalloc(c, &L.tab_own, 13));
                QPAT_HIP(c, hipMemcpyAsync(L.tab_own, tab, sizeof tab, hipMemcpyHostToDevice, c->stream));
                L.tab = L.tab_own;
                QPAT_TRY(dalloc(c, &L.U, 2 * L.N * 14));
                QPAT_TRY(dalloc(c, &L.b, 2 * L.N));
            }
            QPAT_TRY(dalloc(c, &L.dinv, 2 * L.N));
            QPAT_TRY(dalloc(c, &L.x, 2 * L.N));
            QPAT_TRY(dalloc(c, &L.t, 2 * L.N));
            QPAT_TRY(dalloc(c, &L.r, 2 * L.N));
        }
        QPAT_TRY(dalloc(c, &M.w, 2 * nl));
        QPAT_TRY(dalloc(c, &M.gmax, 2 * nl));
        QPAT_TRY(dalloc(c, &M.ainv, 2 * Nc * Nc));
        QPAT_TRY(dalloc(c, &M.pr, 2 * c->N));
        QPAT_TRY(dalloc(c, &M.pp, 2 * c->N));
        QPAT_TRY(dalloc(c, &M.pq, 2 * c->N));
        QPAT_TRY(dalloc(c, &M.parts, 2 * 4 * kMgBlocks));
        QPAT_TRY(dalloc(c, &M.sc, 2));
        QPAT_HIP(c, hipHostMalloc((void**)&M.sc_host, 2 * sizeof(MgScal), hipHostMallocDefault));
        M.lv[0].b = M.pr;   // the V-cycle acts on the PCG residual
    }
    MgState& M = *c->mg;
    const int nl = static_cast<int>(M.lv.size());
    M.lv[0].U = c->MU64;
    for (int l = 0; l + 1 < nl; ++l) {
        const MgLevel& F = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        hipLaunchKernelGGL(k_mg_rap, dim3((unsigned)((C.N + kMgT - 1) / kMgT), 2), dim3(kMgT), 0, c->stream,
                           lv_args(F), C.U, C.nx, C.ny, C.nz);
    }
    QPAT_HIP(c, hipMemsetAsync(M.gmax, 0, 2 * nl * sizeof(uint64_t), c->stream));
    for (int l = 0; l < nl; ++l)
        hipLaunchKernelGGL(k_mg_diag, vgrid(M.lv[l].N), dim3(kMgT), 0, c->stream, lv_args(M.lv[l]), M.lv[l].dinv,
                           M.gmax, nl, l);
    QPAT_HIP(c, hipGetLastError());
    std::vector<uint64_t> gm(2 * nl);
    QPAT_HIP(c, hipMemcpyAsync(gm.data(), M.gmax, gm.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    // coarsest operator to the host for its dense inverse
    const MgLevel& K = M.lv[nl - 1];
    std::vector<double> Uk(2 * K.N * (K.m + 1));
    QPAT_HIP(c, hipMemcpyAsync(Uk.data(), K.U, Uk.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int32_t tabk[4 * 13];
    QPAT_HIP(c, hipMemcpyAsync(tabk, K.tab, sizeof(int32_t) * 4 * K.m, hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<double> w(2 * nl);
    for (int i = 0; i < 2 * nl; ++i) {
        double g;
        std::memcpy(&g, &gm[i], sizeof g);
        if (!(g > 0.0) || !std::isfinite(g)) return fail(c, QPAT_ERR_ARG, "multigrid: non-positive diagonal in M_delta");
        w[i] = 4.0 / (3.0 * g);
    }
    QPAT_HIP(c, hipMemcpyAsync(M.w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const int n = static_cast<int>(K.N), M1 = K.m + 1;
    std::vector<double> inv(2 * (size_t)n * n);
    for (int sys = 0; sys < 2; ++sys) {
        std::vector<double> A((size_t)n * n, 0.0);
        const double* U = Uk.data() + (size_t)sys * n * M1;
        for (int i = 0; i < n; ++i) {
            const int ix = i % K.nx, iy = (i / K.nx) % K.ny, iz = i / (K.nx * K.ny);
            A[(size_t)i * n + i] = U[(size_t)i * M1];
            for (int j = 0; j < K.m; ++j) {
                const int jx = ix + tabk[4 * j], jy = iy + tabk[4 * j + 1], jz = iz + tabk[4 * j + 2];
                if (jx < 0 || jx >= K.nx || jy < 0 || jy >= K.ny || jz < 0 || jz >= K.nz) continue;
                const int k = jx + K.nx * (jy + K.ny * jz);
                A[(size_t)i * n + k] = A[(size_t)k * n + i] = U[(size_t)i * M1 + j + 1];
            }
        }
        if (!spd_inverse(A, n)) return fail(c, QPAT_ERR_ARG, "multigrid: coarsest M_delta is not positive definite");
        std::copy(A.begin(), A.end(), inv.begin() + (size_t)sys * n * n);
    }
    QPAT_HIP(c, hipMemcpyAsync(M.ainv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

// M_delta x = b for both blocks: b in c->b64 [2][N] (overwritten by its
// deflated form), x in c->x64; c->scal[sys].mean receives mean(b)/delta.
qpat_status mg_solve(qpat_ctx* c, SolveStats* st) {
    MgState& M = *c->mg;
    hipStream_t sm = c->stream;
    const dim3 g = vgrid(c->N), one(1, 2);
    // the V-cycle's output buffer is fixed by the sequence of ping-pong swaps
    if (!M.zout) M.zout = vcycle(c, sm, false);
    PcgMg a = pcg_args(c);
    hipLaunchKernelGGL(k_mgp_bstats, g, dim3(kMgT), 0, sm, a, c->b64);
    hipLaunchKernelGGL(k_mgp_init, one, dim3(kMgT), 0, sm, a, c->delta > 0 ? 1.0 / c->delta : 0.0);
    hipLaunchKernelGGL(k_mgp_start, g, dim3(kMgT), 0, sm, a, c->b64);
    QPAT_HIP(c, hipGetLastError());
    auto fetch = [&]() -> qpat_status {
        QPAT_HIP(c, hipMemcpyAsync(M.sc_host, M.sc, 2 * sizeof(MgScal), hipMemcpyDeviceToHost, sm));
        QPAT_HIP(c, hipStreamSynchronize(sm));
        return QPAT_OK;
    };
    for (int restart = 0; restart < 4; ++restart) {
        // first direction of a run: z = V(r), p = z - c
        (void)vcycle(c, sm);
        hipLaunchKernelGGL(k_mgp_dots, g, dim3(kMgT), 0, sm, a);
        hipLaunchKernelGGL(k_mgp_scalars, one, dim3(kMgT), 0, sm, a, 3);
        QPAT_HIP(c, hipGetLastError());
        int chunk = 4;
        for (;;) {
            QPAT_TRY(fetch());
            if (!M.sc_host[0].active && !M.sc_host[1].active) break;
            if (c->opts.use_graphs) {
                char key[96];
                snprintf(key, sizeof key, "%d/%.17g/%d/%d", chunk, a.rtol2, a.maxit, a.deflate);
                auto it = M.graphs.find(key);
                hipGraphExec_t ex = nullptr;
                if (it != M.graphs.end()) {
                    ex = it->second;
                } else {
                    if (!M.cap) QPAT_HIP(c, hipStreamCreateWithFlags(&M.cap, hipStreamNonBlocking));
                    hipGraph_t gr = nullptr;
                    QPAT_HIP(c, hipStreamBeginCapture(M.cap, hipStreamCaptureModeThreadLocal));
                    for (int i = 0; i < chunk; ++i) iteration(c, a, M.cap);
                    QPAT_HIP(c, hipStreamEndCapture(M.cap, &gr));
                    QPAT_HIP(c, hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                    QPAT_HIP(c, hipGraphDestroy(gr));
                    M.graphs[key] = ex;
                }
                QPAT_HIP(c, hipGraphLaunch(ex, sm));
            } else {
                for (int i = 0; i < chunk; ++i) iteration(c, a, sm);
            }
            QPAT_HIP(c, hipGetLastError());
            chunk = std::min(chunk * 2, 16);
        }
        // confirm on the true residual; a failed check restarts from the true residual
        hipLaunchKernelGGL(k_mgp_true, sgrid(c->N), dim3(kMgT), 0, sm, a, c->b64);
        hipLaunchKernelGGL(k_mgp_true_fin, one, dim3(kMgT), 0, sm, a, restart < 3 ? 1 : 0);
        QPAT_HIP(c, hipGetLastError());
        QPAT_TRY(fetch());
        if (!M.sc_host[0].active && !M.sc_host[1].active) break;
    }
    // hand the means to the output kernel of the prior solve
    for (int sys = 0; sys < 2; ++sys) {
        const MgScal& s = M.sc_host[sys];
        QPAT_HIP(c, hipMemcpyAsync(&c->scal[sys].mean, &M.sc[sys].mean, sizeof(double), hipMemcpyDeviceToDevice, sm));
        st->n_solves += 1;
        st->iters_max = std::max(st->iters_max, s.iters);
        st->iters_sum += s.iters;
        const double rel = s.bnorm2 > 0 ? std::sqrt(s.rr / s.bnorm2) : 0.0;
        st->relres_max = std::max(st->relres_max, rel);
        if (!s.done) st->noconv = true;
    }
    return QPAT_OK;
}

}  // namespace qpat
