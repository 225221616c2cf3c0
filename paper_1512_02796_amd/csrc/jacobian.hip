// Forward solve and the matrix-free Jacobian products J s, J^T t.
//
// Appendix: K J^phi = [G(1), G(2)] with G(1)_ij = -int phi_j grad(phi).grad(phi_i),
// G(2)_ij = -int phi_j phi phi_i, and
//   J s   = diag(mu) K^{-1} (G(1) diag(kappa) s1 + G(2) diag(mu) s2) + diag(phi) diag(mu) s2
//   J^T t = [diag(kappa) G(1)^T K^{-1} diag(mu) t ; diag(mu) (G(2) K^{-1} diag(mu) t + diag(phi) t)].
// G is never formed. K is linear in the nodal coefficients, so for P1 fields
//   G(1) u1 + G(2) u2 = -(S(u1) + Mass(u2)) phi            (same element loop as K)
//   (G(1)^T z)_j      = -sum_{T at j} |T|/4 grad(phi_T).grad(z_T)
//   G(2) z            = -Mass(phi) z
// with S(u)_ab = mean_T(u) |T| grad(l_a).grad(l_b) and
// Mass(u)_ab = |T| (1 + d_ab) (sum_T u + u_a + u_b) / 120.
// Data-space vectors inside the library are interleaved [N][n_pad]; the
// illuminations are solved in blocks of B right-hand sides. J s: on lattice
// meshes S(u1) + Mass(u2) is assembled once per product in the stencil form
// and applied to each block by the tiled stencil kernel; elsewhere a node
// loop over the adjacent elements per block. J^T t: the G^T terms are summed
// per element over the blocks, then gathered per node.
#include "qpat_internal.h"

namespace qpat {
namespace {

struct Geo4 {
    double vol;
    double g[4][3];
};

// per-tetrahedron geometry, or its class in a small table (qpat_ctx::geo_cls)
struct GeoRef {
    const double* geo;
    const uint8_t* cls;   // null: no classes
    const double* tab;
};

__device__ __forceinline__ void load_geo4(const double* __restrict__ geo, int32_t e, Geo4& G) {
    const double* p = geo + (int64_t)kTetGeo * e;
    G.vol = p[0];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        G.g[1][d] = p[1 + d];
        G.g[2][d] = p[4 + d];
        G.g[3][d] = p[7 + d];
        G.g[0][d] = -(G.g[1][d] + G.g[2][d] + G.g[3][d]);
    }
}

__device__ __forceinline__ void load_geo4(const GeoRef& r, int32_t e, Geo4& G) {
    if (r.cls)
        load_geo4(r.tab, static_cast<int32_t>(r.cls[e]), G);
    else
        load_geo4(r.geo, e, G);
}

// right-hand sides handled by one thread of the G kernels: the per-tetrahedron
// geometry and coefficients are loaded once for all of them
template <int B>
constexpr int kGroup = B > 8 ? 8 : B;

// b[row][k] = -(S(u1) + Mass(u2)) phi_{col0+k}, u1 = kappa s1, u2 = mu s2.
// Per tetrahedron at row vertex a the contribution is linear in the vertex
// values of phi: sum_c w_c phi_c with
//   w_c = mean(u1) |T| grad(l_a).grad(l_c) + |T| (1 + d_ac) (sum u2 + u2_a + u2_c) / 120.
template <int B>
__global__ __launch_bounds__(kThreads) void k_gfwd(int64_t N, const int32_t* __restrict__ tets,
                                                  const double* __restrict__ geo, const int32_t* __restrict__ n2t_ptr,
                                                  const int32_t* __restrict__ n2t, const double* __restrict__ kappa,
                                                  const double* __restrict__ mu, const double* __restrict__ s,
                                                  const double* __restrict__ phi, int n_pad, int col0,
                                                  double* __restrict__ b) {
    constexpr int KG = kGroup<B>, G = B / KG;
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * G) return;
    const int64_t row = t / G;
    const int k0 = static_cast<int>(t % G) * KG;
    double acc[KG];
#pragma unroll
    for (int i = 0; i < KG; ++i) acc[i] = 0.0;
    for (int32_t q = n2t_ptr[row]; q < n2t_ptr[row + 1]; ++q) {
        const int32_t e = n2t[q] >> 2, a = n2t[q] & 3;
        Geo4 G4;
        load_geo4(geo, e, G4);
        int32_t v[4];
        double u1 = 0.0, u2[4], s2 = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = tets[4 * e + c];
            u1 += kappa[v[c]] * s[v[c]];
            u2[c] = mu[v[c]] * s[N + v[c]];
            s2 += u2[c];
        }
        u1 *= 0.25;
        double ga[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int c = 0; c < 4; ++c)   // select with compile-time indices: no scratch copy
#pragma unroll
            for (int d = 0; d < 3; ++d) ga[d] = c == a ? G4.g[c][d] : ga[d];   // runtime vertex: select once
        double w[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double gg = ga[0] * G4.g[c][0] + ga[1] * G4.g[c][1] + ga[2] * G4.g[c][2];
            w[c] = u1 * G4.vol * gg + G4.vol * (1.0 / 120.0) * (c == a ? 2.0 : 1.0) * (s2 + u2[a] + u2[c]);
        }
#pragma unroll
        for (int i = 0; i < KG; ++i) {
            const int kk = col0 + k0 + i;
            double sum = 0.0;
#pragma unroll
            for (int c = 0; c < 4; ++c) sum += w[c] * phi[(int64_t)v[c] * n_pad + kk];
            acc[i] -= sum;
        }
    }
#pragma unroll
    for (int i = 0; i < KG; ++i) b[row * B + k0 + i] = acc[i];
}

// ---- lattice meshes: the same products through the stencil form
// dK(s) = S(kappa s1) + Mass(mu s2) in the stencil form of the lattice
// (diagonal and upper offsets, [N][m+1]): the element sums of the assembly of
// K without the boundary term, so G(1) diag(kappa) s1 + G(2) diag(mu) s2 =
// -dK(s) phi for every illumination, one stencil product per block.
// kSplit consecutive threads share a node's element list (one element in
// kSplit each) and sum by shuffles: the list's loads are independent, so
// more of them are in flight than with one thread per node.
constexpr int kSplit = 8;

// the coefficients of dK(s) per node: uu[i] = (kappa_i s1_i, mu_i s2_i)
__global__ __launch_bounds__(kThreads) void k_dk_coef(int64_t N, const double* __restrict__ kappa,
                                                      const double* __restrict__ mu, const double* __restrict__ s,
                                                      double* __restrict__ uu) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    uu[2 * i] = kappa[i] * s[i];
    uu[2 * i + 1] = mu[i] * s[N + i];
}

// M1: stored entries per row (8 on the Kuhn lattice, else kMaxUpper + 1)
template <int M1>
__global__ __launch_bounds__(kThreads) void k_dk_lattice(int64_t N, Lattice lat, const int32_t* __restrict__ tets,
                                                         GeoRef geo,
                                                         const int32_t* __restrict__ n2t_ptr,
                                                         const int32_t* __restrict__ n2t,
                                                         const double* __restrict__ uu, double* __restrict__ U) {
    // Node order: the blocks of XCD x (block b runs on XCD b mod 8) take the
    // y-strip [x ny / 8, (x + 1) ny / 8) of every plane (z-slabs when ny < 8)
    // plane by plane, so the elements around the strip's planes stay in that
    // XCD's L2 while the four nodes of each element read them.
    const int64_t nx = lat.nx, ny = lat.ny, nxy = nx * ny;
    const int xcd = blockIdx.x & 7;
    int64_t y0 = 0, ys = ny, z0 = 0, zs = lat.nz;
    if (ny >= 8) {
        y0 = xcd * ny / 8;
        ys = (xcd + 1) * ny / 8 - y0;
    } else {
        z0 = xcd * lat.nz / 8;
        zs = (xcd + 1) * (int64_t)lat.nz / 8 - z0;
    }
    const int64_t span = nx * ys * zs;
    const int part = threadIdx.x % kSplit;
    const int64_t gpb = kThreads / kSplit, per = (gridDim.x >> 3) * gpb;
    // neighbour offsets: with nx, ny >= 3 the linear offset of a neighbour at
    // most one step away per axis determines (dx, dy, dz) by comparisons
    const bool fast = lat.nx >= 3 && lat.ny >= 3;
    for (int64_t n0 = (blockIdx.x >> 3) * gpb; n0 < span; n0 += per) {   // uniform over the block
    const int64_t n = n0 + threadIdx.x / kSplit;
    const bool valid = n < span;   // whole groups of kSplit lanes
    const int rx = static_cast<int>(n % nx);
    const int ry = static_cast<int>(y0 + (n / nx) % ys), rz = static_cast<int>(z0 + n / (nx * ys));
    const int64_t row = rx + nx * (ry + ny * (int64_t)rz);
    double acc[M1];
#pragma unroll
    for (int j = 0; j < M1; ++j) acc[j] = 0.0;
    const int32_t q0 = valid ? n2t_ptr[row] : 0, q1 = valid ? n2t_ptr[row + 1] : 0;
    for (int32_t q = q0 + part; q < q1; q += kSplit) {
        const int32_t e = n2t[q] >> 2, a = n2t[q] & 3;
        Geo4 G4;
        load_geo4(geo, e, G4);
        int32_t v[4];
        double u1 = 0.0, u2[4], s2 = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            v[c] = tets[4 * e + c];
            const double2 w2 = *reinterpret_cast<const double2*>(uu + 2 * (int64_t)v[c]);
            u1 += w2.x;
            u2[c] = w2.y;
            s2 += u2[c];
        }
        u1 *= 0.25;
        double ga[3] = {0.0, 0.0, 0.0}, u2a = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c == a) u2a = u2[c];
#pragma unroll
        for (int c = 0; c < 4; ++c)   // select with compile-time indices: no scratch copy
#pragma unroll
            for (int d = 0; d < 3; ++d) ga[d] = c == a ? G4.g[c][d] : ga[d];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const double gg = ga[0] * G4.g[c][0] + ga[1] * G4.g[c][1] + ga[2] * G4.g[c][2];
            const double w = u1 * G4.vol * gg + G4.vol * (1.0 / 120.0) * (c == a ? 2.0 : 1.0) * (s2 + u2a + u2[c]);
            int dx, dy, dz;
            if (fast) {
                int64_t lin = v[c] - row;
                dz = lin > nxy / 2 ? 1 : (lin < -nxy / 2 ? -1 : 0);
                lin -= dz * nxy;
                dy = lin > nx / 2 ? 1 : (lin < -nx / 2 ? -1 : 0);
                dx = static_cast<int>(lin - dy * nx);
            } else {
                const int64_t vc = v[c];
                dx = static_cast<int>(vc % nx) - rx;
                dy = static_cast<int>((vc / nx) % lat.ny) - ry;
                dz = static_cast<int>(vc / nxy) - rz;
            }
            const int slot = lat.code[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];   // -1: a lower entry
#pragma unroll
            for (int j = 0; j < M1; ++j) acc[j] += slot == j ? w : 0.0;
        }
    }
#pragma unroll
    for (int j = 0; j < M1; ++j)
#pragma unroll
        for (int off = kSplit / 2; off >= 1; off >>= 1) acc[j] += __shfl_xor(acc[j], off);
    if (valid && part == 0)
        for (int j = 0; j < lat.m + 1; ++j) U[row * (lat.m + 1) + j] = acc[j];
    }
}

// J^T t, element by element: per tetrahedron and block of illuminations,
//   tq[T]   (+)= sum_k |T|/4 grad(phi_k).grad(z_k)
//   tr[T][a] (+)= sum_k (Mass_T(phi_k) z_k)_a,
// KT right-hand sides per thread, the B / KT threads of a tetrahedron summing
// by shuffles. first: overwrite (first block) instead of accumulating.
template <int B>
constexpr int kTetRhs = B >= 4 ? 4 : B;

template <int B>
__global__ __launch_bounds__(kThreads) void k_gadj_tet(int64_t E, const int32_t* __restrict__ tets,
                                                       GeoRef geo, const double* __restrict__ phi,
                                                       int n_pad, int col0, const double* __restrict__ z, int first,
                                                       double* __restrict__ tq, double* __restrict__ tr) {
    constexpr int KT = kTetRhs<B>, G = B / KT;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool valid = t < E * G;
    const int64_t e = valid ? t / G : 0;
    const int k0 = static_cast<int>(t % G) * KT;
    double q = 0.0, r[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
        Geo4 G4;
        load_geo4(geo, static_cast<int32_t>(e), G4);
        int32_t v[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) v[c] = tets[4 * e + c];
#pragma unroll
        for (int i = 0; i < KT; ++i) {
            double ph[4], zz[4], sp = 0.0, gp[3] = {0.0, 0.0, 0.0}, gz[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                ph[c] = phi[(int64_t)v[c] * n_pad + col0 + k0 + i];
                zz[c] = z[(int64_t)v[c] * B + k0 + i];
                sp += ph[c];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    gp[d] += ph[c] * G4.g[c][d];
                    gz[d] += zz[c] * G4.g[c][d];
                }
            }
            q += 0.25 * G4.vol * (gp[0] * gz[0] + gp[1] * gz[1] + gp[2] * gz[2]);
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double m = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) m += (c == a ? 2.0 : 1.0) * (sp + ph[a] + ph[c]) * zz[c];
                r[a] += G4.vol * (1.0 / 120.0) * m;
            }
        }
    }
#pragma unroll
    for (int off = G >> 1; off >= 1; off >>= 1) {
        q += __shfl_xor(q, off);
#pragma unroll
        for (int a = 0; a < 4; ++a) r[a] += __shfl_xor(r[a], off);
    }
    if (valid && k0 == 0) {
        if (first) {
            tq[e] = q;
#pragma unroll
            for (int a = 0; a < 4; ++a) tr[4 * e + a] = r[a];
        } else {
            tq[e] += q;
#pragma unroll
            for (int a = 0; a < 4; ++a) tr[4 * e + a] += r[a];
        }
    }
}

// a1[row] = -sum_{T at row} tq[T], a2[row] = -sum_{T at row} tr[T][a] + sum_k phi_k,row t_k,row
// (tmode 0: t external [n_ill][N]; tmode 1: t = W u interleaved [N][n_pad])
__global__ __launch_bounds__(kThreads) void k_gadj_gather(int64_t N, const int32_t* __restrict__ n2t_ptr,
                                                          const int32_t* __restrict__ n2t,
                                                          const double* __restrict__ tq,
                                                          const double* __restrict__ tr,
                                                          const double* __restrict__ phi, int n_pad, int n_ill,
                                                          int tmode, const double* __restrict__ t_ext,
                                                          const double* __restrict__ W, const double* __restrict__ U,
                                                          double* __restrict__ a1, double* __restrict__ a2) {
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = t / kSplit;
    const int part = static_cast<int>(t % kSplit);
    const bool valid = row < N;   // whole groups of kSplit lanes
    double s1 = 0.0, s2 = 0.0;
    if (valid) {
        for (int32_t q = n2t_ptr[row] + part; q < n2t_ptr[row + 1]; q += kSplit) {
            const int32_t e = n2t[q] >> 2, a = n2t[q] & 3;
            s1 -= tq[e];
            s2 -= tr[4 * (int64_t)e + a];
        }
        for (int kk = part; kk < n_ill; kk += kSplit) {
            const double tv = tmode == 0 ? t_ext[(int64_t)kk * N + row] : W[row * n_pad + kk] * U[row * n_pad + kk];
            s2 += phi[row * n_pad + kk] * tv;
        }
    }
#pragma unroll
    for (int off = kSplit / 2; off >= 1; off >>= 1) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    if (valid && part == 0) {
        a1[row] = s1;
        a2[row] = s2;
    }
}

// solver block <- columns col0..col0+B-1 of an interleaved data array
template <int B>
__global__ void k_pack(int64_t N, const double* __restrict__ src, int n_pad, int col0, double* __restrict__ dst) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * B) return;
    dst[t] = src[(t / B) * n_pad + col0 + (t % B)];
}

template <int B>
__global__ void k_unpack(int64_t N, const double* __restrict__ src, int n_pad, int col0, double* __restrict__ dst) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * B) return;
    dst[(t / B) * n_pad + col0 + (t % B)] = src[t];
}

// solver block <- columns col0..col0+B-1 of a caller array [n_ill][N] (zero past n_ill)
template <int B>
__global__ void k_pack_ext(int64_t N, const double* __restrict__ src, int n_ill, int col0, double* __restrict__ dst) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * B) return;
    const int kk = col0 + static_cast<int>(t % B);
    dst[t] = kk < n_ill ? src[(int64_t)kk * N + t / B] : 0.0;
}

// adjoint right-hand side b = mu t (tmode 0: external t; 1: t = W u interleaved)
template <int B>
__global__ void k_adj_rhs(int64_t N, const double* __restrict__ mu, int n_pad, int n_ill, int col0, int tmode,
                          const double* __restrict__ t_ext, const double* __restrict__ W,
                          const double* __restrict__ U, double* __restrict__ b) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * B) return;
    const int64_t row = t / B;
    const int kk = col0 + static_cast<int>(t % B);
    double tv = 0.0;
    if (kk < n_ill) {
        if (tmode == 0) tv = t_ext[(int64_t)kk * N + row];
        else tv = W[row * n_pad + kk] * U[row * n_pad + kk];
    }
    b[t] = mu[row] * tv;
}

// J s output: y = mu w + phi mu s2.
// mode 0: out [n_ill][N]; mode 1: q = W y - alpha u (interleaved); mode 2: out interleaved y
template <int B>
__global__ void k_jvp_out(int64_t N, const double* __restrict__ mu, const double* __restrict__ phi,
                          const double* __restrict__ s, const double* __restrict__ w, int n_pad, int n_ill, int col0,
                          int mode, double* __restrict__ out, const double* __restrict__ W,
                          const double* __restrict__ U, const LsqrScal* __restrict__ ls) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= N * B) return;
    const int64_t row = t / B;
    const int kk = col0 + static_cast<int>(t % B);
    const int64_t di = row * n_pad + kk;
    const double y = mu[row] * (w[t] + phi[di] * s[N + row]);
    if (mode == 0) {
        if (kk < n_ill) out[(int64_t)kk * N + row] = y;
    } else if (mode == 1) {
        out[di] = (kk < n_ill ? W[di] * y : 0.0) - ls->alpha * U[di];
    } else {
        out[di] = kk < n_ill ? y : 0.0;
    }
}

// J^T t output: out = [kappa a1 ; mu a2] (- beta what when sub)
__global__ void k_vjp_out(int64_t N, const double* __restrict__ kappa, const double* __restrict__ mu,
                          const double* __restrict__ a1, const double* __restrict__ a2, double* __restrict__ out,
                          int sub, const double* __restrict__ wh, const LsqrScal* __restrict__ ls) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double o1 = kappa[i] * a1[i], o2 = mu[i] * a2[i];
    if (sub) {
        const double b = ls->beta;
        o1 -= b * wh[i];
        o2 -= b * wh[N + i];
    }
    out[i] = o1;
    out[N + i] = o2;
}

int block_size(const qpat_ctx* c) {
    int B = c->opts.max_rhs_block;
    return B < c->n_pad ? B : c->n_pad;
}

#define QPAT_DISPATCH_B(B, CALL)                                  \
    switch (B) {                                                  \
        case 1: { constexpr int BB = 1; CALL; } break;            \
        case 2: { constexpr int BB = 2; CALL; } break;            \
        case 4: { constexpr int BB = 4; CALL; } break;            \
        case 8: { constexpr int BB = 8; CALL; } break;            \
        case 16: { constexpr int BB = 16; CALL; } break;          \
        default: return fail(c, QPAT_ERR_ARG, "bad block size"); \
    }

}  // namespace

// K x = b for one block of B right-hand sides: multigrid-preconditioned PCG
// where its hierarchy is built, Jacobi-PCG otherwise
inline GeoRef geo_ref(const qpat_ctx* c) { return GeoRef{c->geo, c->geo_cls, c->geo_tab}; }

static qpat_status k_solve(qpat_ctx* c, int B, SolveStats* st, bool has_x0 = false) {
    if (mg_ready(c, Op::K)) return mg_solve(c, Op::K, B, st, has_x0);
    return pcg_solve(c, Op::K, B, st, has_x0);
}

qpat_status forward_solve(qpat_ctx* c, SolveStats* st) {
    const int B = block_size(c);
    const dim3 g(grid_for(c->N * B, kThreads, 1 << 30)), blk(kThreads);
    for (int col0 = 0; col0 < c->n_pad; col0 += B) {
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_pack<BB>, g, blk, 0, c->stream, c->N, c->f, c->n_pad, col0, c->b64));
        QPAT_TRY(k_solve(c, B, st));
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_unpack<BB>, g, blk, 0, c->stream, c->N, c->x64, c->n_pad, col0, c->phi));
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// forward solves started from a caller's initial guess x0 [n_ill][N]
qpat_status forward_solve_x0(qpat_ctx* c, const double* x0, SolveStats* st) {
    const int B = block_size(c);
    const dim3 g(grid_for(c->N * B, kThreads, 1 << 30)), blk(kThreads);
    for (int col0 = 0; col0 < c->n_pad; col0 += B) {
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_pack<BB>, g, blk, 0, c->stream, c->N, c->f, c->n_pad, col0, c->b64));
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_pack_ext<BB>, g, blk, 0, c->stream, c->N, x0, c->n_ill, col0, c->x64));
        QPAT_TRY(k_solve(c, B, st, true));
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_unpack<BB>, g, blk, 0, c->stream, c->N, c->x64, c->n_pad, col0, c->phi));
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status jvp_core(qpat_ctx* c, const double* s, int mode, double* out, SolveStats* st) {
    const int B = block_size(c);
    const dim3 g(grid_for(c->N * B, kThreads, 1 << 30)), blk(kThreads);
    // lattice meshes: dK(s) once in the stencil form, then one tiled stencil
    // product per block (else the element loop per block)
    const bool lat = c->lat.on && c->opts.operator_format == 1 && B >= 8;
    if (lat) {
        if (!c->dK) {
            QPAT_TRY(dalloc(c, &c->dK, (int64_t)(c->lat.m + 1) * c->N));
            QPAT_TRY(dalloc(c, &c->dKc, 2 * c->N));
        }
        hipLaunchKernelGGL(k_dk_coef, dim3(grid_for(c->N, kThreads, 1 << 30)), blk, 0, c->stream, c->N, c->kappa, c->mu,
                           s, c->dKc);
        // a multiple of 8 blocks (the XCD strips), several per compute unit
        const dim3 gd((std::min<int64_t>((c->N * kSplit + kThreads - 1) / kThreads, 4096) + 7) & ~7);
        if (c->lat.m == 7)
            hipLaunchKernelGGL(k_dk_lattice<8>, gd, blk, 0, c->stream, c->N, c->lat, c->tets, geo_ref(c), c->n2t_ptr,
                               c->n2t, c->dKc, c->dK);
        else
            hipLaunchKernelGGL(k_dk_lattice<kMaxUpper + 1>, gd, blk, 0, c->stream, c->N, c->lat, c->tets, geo_ref(c),
                               c->n2t_ptr, c->n2t, c->dKc, c->dK);
    }
    for (int col0 = 0; col0 < c->n_pad; col0 += B) {
        bool done = false;
        if (lat) QPAT_TRY(mg_stencil_apply(c, B, c->dK, c->phi, c->n_pad, col0, c->b64, -1.0, &done));
        if (!done)
            QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_gfwd<BB>,
                                                  dim3(grid_for(c->N * (BB / kGroup<BB>), kThreads, 1 << 30)), blk, 0,
                                                  c->stream, c->N, c->tets, c->geo, c->n2t_ptr, c->n2t, c->kappa,
                                                  c->mu, s, c->phi, c->n_pad, col0, c->b64));
        QPAT_TRY(k_solve(c, B, st));
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_jvp_out<BB>, g, blk, 0, c->stream, c->N, c->mu, c->phi, s, c->x64,
                                              c->n_pad, c->n_ill, col0, mode, out, c->lw, c->lu, c->ls));
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// mode 0: t external [n_ill][N], out = J^T t
// mode 1: t = W u (c->lw, c->lu), out = J^T t
// mode 2: as 1, out = J^T t - beta what
// The G^T terms are summed per tetrahedron over the blocks of illuminations,
// then gathered per node once.
qpat_status vjp_core(qpat_ctx* c, const double* t, int mode, double* out, SolveStats* st) {
    const int B = block_size(c);
    const dim3 g(grid_for(c->N * B, kThreads, 1 << 30)), blk(kThreads);
    const int tmode = mode == 0 ? 0 : 1;
    if (!c->tq) {
        QPAT_TRY(dalloc(c, &c->tq, c->E));
        QPAT_TRY(dalloc(c, &c->tr, 4 * c->E));
    }
    for (int col0 = 0; col0 < c->n_pad; col0 += B) {
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_adj_rhs<BB>, g, blk, 0, c->stream, c->N, c->mu, c->n_pad, c->n_ill,
                                              col0, tmode, t, c->lw, c->lu, c->b64));
        QPAT_TRY(k_solve(c, B, st));
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_gadj_tet<BB>,
                                              dim3(grid_for(c->E * (BB / kTetRhs<BB>), kThreads, 1 << 30)), blk, 0,
                                              c->stream, c->E, c->tets, geo_ref(c), c->phi, c->n_pad, col0, c->x64,
                                              col0 == 0 ? 1 : 0, c->tq, c->tr));
    }
    hipLaunchKernelGGL(k_gadj_gather, dim3(grid_for(c->N * kSplit, kThreads, 1 << 30)), blk, 0, c->stream, c->N, c->n2t_ptr,
                       c->n2t, c->tq, c->tr, c->phi, c->n_pad, c->n_ill, tmode, t, c->lw, c->lu, c->acc1, c->acc2);
    hipLaunchKernelGGL(k_vjp_out, dim3(grid_for(c->N, kThreads, 1 << 30)), blk, 0, c->stream, c->N, c->kappa, c->mu,
                       c->acc1, c->acc2, out, mode == 2 ? 1 : 0, c->lwh, c->ls);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

}  // namespace qpat
