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
#include <cstring>

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

// ------------------------------------------------------------- voxel form
// On a Kuhn lattice of equal voxels (spacings h_x, h_y, h_z) every element is
// a path tetrahedron of its voxel: corners 0 -> b1 -> b1|b2 -> 7 for a
// permutation (s1, s2, s3) of the axes (corner bit 1 << axis). Its
// barycentric gradients are steps along the path: grad l_0 = -e1/h1,
// grad l_m = e_m/h_m - e_(m+1)/h_(m+1), grad l_3 = e3/h3 (e_m the unit vector
// of axis s_m, h_m its spacing). Hence |T| grad l_p . grad l_q is tridiagonal
// in path order (w_m = 1/h_m^2):
//   (p, p): w_1, w_1 + w_2, w_2 + w_3, w_3;  (p, p + 1): -w_(p+1);  else 0,
// and grad f . grad g = sum_m (f_m - f_(m-1)) (g_m - g_(m-1)) w_m. |T| = h_x h_y h_z / 6.
// The kernels below read only node values: no element lists, connectivity
// or per-element geometry.
struct VoxGeo {
    double w[3];         // 1 / h^2 along x, y, z
    double vol;          // |T|
};
constexpr int kPerm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};

// dK(s) rows [N][8] from uu = (kappa s1, mu s2), one thread per node: the 27
// neighbour values in registers, then the path tetrahedra through the node in
// each of its 8 voxels (the node is corner c of the voxel at node - bits(c)),
// with every index fixed at compile time. On the Kuhn pattern the slot of
// upper offset mask m (x = 1, y = 2, z = 4) is m itself.
template <int C, int T, int Q>
__device__ __forceinline__ void dk_term(double (&acc)[8], const double (&a1)[27], const double (&a2)[27],
                                        const VoxGeo& vg, bool vin) {
    constexpr int s0 = kPerm[T][0], s1 = kPerm[T][1], s2 = kPerm[T][2];
    constexpr int P[4] = {0, 1 << s0, (1 << s0) | (1 << s1), 7};
    constexpr int pos = C == P[0] ? 0 : C == P[1] ? 1 : C == P[2] ? 2 : C == P[3] ? 3 : -1;
    if constexpr (pos >= 0 && Q >= pos) {
        // neighbour slot of voxel corner k: offset bits(k) - bits(C) in {-1, 0, 1}^3
        auto nb = [](int k) constexpr {
            return ((k & 1) - (C & 1) + 1) + 3 * (((k >> 1) & 1) - ((C >> 1) & 1) + 1) + 9 * ((k >> 2) - (C >> 2) + 1);
        };
        constexpr int n0 = nb(P[0]), n1 = nb(P[1]), n2 = nb(P[2]), n3 = nb(P[3]), nq = nb(P[Q]);
        const double u1 = 0.25 * (a1[n0] + a1[n1] + a1[n2] + a1[n3]);
        const double ss = a2[n0] + a2[n1] + a2[n2] + a2[n3];
        const double wm[3] = {vg.w[s0], vg.w[s1], vg.w[s2]};
        double g;
        if constexpr (Q == pos)
            g = pos == 0 ? wm[0] : pos == 1 ? wm[0] + wm[1] : pos == 2 ? wm[1] + wm[2] : wm[2];
        else if constexpr (Q == pos + 1)
            g = -(pos == 0 ? wm[0] : pos == 1 ? wm[1] : wm[2]);
        else
            g = 0.0;
        const double val = u1 * vg.vol * g + vg.vol * (1.0 / 120.0) * (Q == pos ? 2.0 : 1.0) * (ss + a2[13] + a2[nq]);
        acc[P[Q] ^ C] += vin ? val : 0.0;
    }
}
template <int C, int... TQ>
__device__ __forceinline__ void dk_corner(double (&acc)[8], const double (&a1)[27], const double (&a2)[27],
                                          const VoxGeo& vg, bool vin, std::integer_sequence<int, TQ...>) {
    (dk_term<C, TQ / 4, TQ % 4>(acc, a1, a2, vg, vin), ...);
}

__global__ __launch_bounds__(kThreads) void k_dk_voxel(int64_t N, Lattice lat, VoxGeo vg,
                                                       const double* __restrict__ uu, double* __restrict__ U) {
    const int64_t nx = lat.nx, ny = lat.ny, nxy = nx * ny;
    const int xcd = blockIdx.x & 7;   // the XCD strips of k_dk_lattice
    int64_t y0 = 0, ys = ny, z0 = 0, zs = lat.nz;
    if (ny >= 8) {
        y0 = xcd * ny / 8;
        ys = (xcd + 1) * ny / 8 - y0;
    } else {
        z0 = xcd * lat.nz / 8;
        zs = (xcd + 1) * (int64_t)lat.nz / 8 - z0;
    }
    const int64_t span = nx * ys * zs;
    const int64_t per = (gridDim.x >> 3) * (int64_t)kThreads;
    const double2* uu2 = reinterpret_cast<const double2*>(uu);
    for (int64_t n = (blockIdx.x >> 3) * (int64_t)kThreads + threadIdx.x; n < span; n += per) {
        const int rx = static_cast<int>(n % nx);
        const int ry = static_cast<int>(y0 + (n / nx) % ys), rz = static_cast<int>(z0 + n / (nx * ys));
        const int64_t row = rx + nx * (ry + ny * (int64_t)rz);
        double a1[27], a2[27];
#pragma unroll
        for (int q = 0; q < 27; ++q) {   // clamped: values outside the lattice only meet outside voxels
            const int x = min(max(rx + q % 3 - 1, 0), lat.nx - 1);
            const int y = min(max(ry + (q / 3) % 3 - 1, 0), lat.ny - 1);
            const int z = min(max(rz + q / 9 - 1, 0), lat.nz - 1);
            const double2 w2 = uu2[x + nx * (y + ny * (int64_t)z)];
            a1[q] = w2.x;
            a2[q] = w2.y;
        }
        double acc[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) acc[j] = 0.0;
        auto in = [&](int c) {   // the voxel in which the node is corner c
            const int vx = rx - (c & 1), vy = ry - ((c >> 1) & 1), vz = rz - (c >> 2);
            return vx >= 0 && vx < lat.nx - 1 && vy >= 0 && vy < lat.ny - 1 && vz >= 0 && vz < lat.nz - 1;
        };
        using S = std::make_integer_sequence<int, 24>;
        dk_corner<0>(acc, a1, a2, vg, in(0), S{});
        dk_corner<1>(acc, a1, a2, vg, in(1), S{});
        dk_corner<2>(acc, a1, a2, vg, in(2), S{});
        dk_corner<3>(acc, a1, a2, vg, in(3), S{});
        dk_corner<4>(acc, a1, a2, vg, in(4), S{});
        dk_corner<5>(acc, a1, a2, vg, in(5), S{});
        dk_corner<6>(acc, a1, a2, vg, in(6), S{});
        dk_corner<7>(acc, a1, a2, vg, in(7), S{});
#pragma unroll
        for (int j = 0; j < 8; ++j) U[row * 8 + j] = acc[j];
    }
}

// J^T t per voxel and right-hand side k (B lanes per voxel), summed over the
// lanes: QR[c][v] (+)= sum over the voxel's tetrahedra T at corner c of
// sum_k |T|/4 grad(phi_k).grad(z_k), and QR[8 + c][v] of sum_k (Mass_T(phi_k) z_k)_c
// (entry-major, so that the node gather reads consecutive voxels).
template <int T>
__device__ __forceinline__ void gadj_tet_terms(double (&Q)[8], double (&R)[8], const double (&f)[8],
                                               const double (&g)[8], const VoxGeo& vg) {
    constexpr int s0 = kPerm[T][0], s1 = kPerm[T][1], s2 = kPerm[T][2];
    constexpr int P0 = 0, P1 = 1 << s0, P2 = (1 << s0) | (1 << s1), P3 = 7;
    // grad f . grad g (the factor |T| / 4 is applied once per corner at the end)
    const double q = vg.w[s0] * (f[P1] - f[P0]) * (g[P1] - g[P0]) + vg.w[s1] * (f[P2] - f[P1]) * (g[P2] - g[P1]) +
                     vg.w[s2] * (f[P3] - f[P2]) * (g[P3] - g[P2]);
    const double sp = f[P0] + f[P1] + f[P2] + f[P3];
    const double sz = g[P0] + g[P1] + g[P2] + g[P3];
    const double cc = sp * sz + (f[P0] * g[P0] + f[P1] * g[P1] + f[P2] * g[P2] + f[P3] * g[P3]);
    // sum_c (1 + d_ac)(sp + f_a + f_c) z_c = (sp + f_a) sz + pz + (sp + 2 f_a) z_a
    //   = cc + f_a (sz + 2 z_a) + sp z_a  (the factor |T| / 120 at the end)
    auto add = [&](auto AA) {
        constexpr int A = decltype(AA)::value;
        Q[A] += q;
        R[A] += cc + f[A] * (sz + 2.0 * g[A]) + sp * g[A];
    };
    add(std::integral_constant<int, P0>{});
    add(std::integral_constant<int, P1>{});
    add(std::integral_constant<int, P2>{});
    add(std::integral_constant<int, P3>{});
}

// one halving step of the lane sum: offset O, H values kept of 2 H
template <int O, int H>
__device__ __forceinline__ void halve(double (&e)[16], bool hi) {
#pragma unroll
    for (int i = 0; i < H; ++i) {
        const double send = hi ? e[i] : e[i + H];
        const double keep = hi ? e[i + H] : e[i];
        e[i] = keep + __shfl_xor(send, O);
    }
}
template <int B, int O>
__device__ __forceinline__ void halve_all(double (&e)[16], int k) {
    if constexpr (O >= 1) {
        halve<O, 16 * O / B>(e, (k & O) != 0);
        halve_all<B, O / 2>(e, k);
    }
}

template <int B>
__global__ __launch_bounds__(kThreads) void k_gadj_vox(Lattice lat, VoxGeo vg, const double* __restrict__ phi,
                                                       int n_pad, int col0, const double* __restrict__ z, int first,
                                                       double* __restrict__ QR) {
    // 32-bit offsets throughout (the set-up admits this form only where every
    // array fits them): voxel coordinates by 32-bit divisions, corner offsets
    // uniform over the block
    const uint32_t nx = lat.nx, ny = lat.ny, nxy = nx * ny;
    const uint32_t vxn = nx - 1, vyn = ny - 1, vxyn = vxn * vyn, Nv = vxyn * (lat.nz - 1);
    // block b runs on XCD b mod 8: each XCD takes a contiguous eighth of the
    // voxels, so the corner values shared along y and z stay in its L2
    const uint32_t per_xcd = (Nv + 7) / 8;
    const uint32_t loc = (blockIdx.x >> 3) * (kThreads / B) + threadIdx.x / B;
    const uint32_t v = (blockIdx.x & 7) * per_xcd + loc;
    const int k = static_cast<int>(threadIdx.x % B);
    const bool valid = loc < per_xcd && v < Nv;   // whole groups of B lanes
    double Q[8], R[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) Q[c] = R[c] = 0.0;
    if (valid) {
        const uint32_t vx = v % vxn, vy = (v / vxn) % vyn, vz = v / vxyn;
        const uint32_t n0 = vx + nx * (vy + ny * vz);
        const uint32_t N = nxy * lat.nz;
        const auto bp = rsrc(phi, N * static_cast<uint32_t>(n_pad) * 8u);
        const auto bz = rsrc(z, N * static_cast<uint32_t>(B) * 8u);
        const uint32_t p0 = (n0 * static_cast<uint32_t>(n_pad) + static_cast<uint32_t>(col0 + k)) * 8u;
        const uint32_t z0 = (n0 * B + k) * 8u;
        double f[8], g[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t cn = (c & 1) + nx * ((c >> 1) & 1) + nxy * (c >> 2);   // uniform
            f[c] = bload<double>(bp, p0 + cn * static_cast<uint32_t>(n_pad) * 8u);
            g[c] = bload<double>(bz, z0 + cn * (B * 8u));
        }
        gadj_tet_terms<0>(Q, R, f, g, vg);
        gadj_tet_terms<1>(Q, R, f, g, vg);
        gadj_tet_terms<2>(Q, R, f, g, vg);
        gadj_tet_terms<3>(Q, R, f, g, vg);
        gadj_tet_terms<4>(Q, R, f, g, vg);
        gadj_tet_terms<5>(Q, R, f, g, vg);
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            Q[c] *= 0.25 * vg.vol;
            R[c] *= vg.vol * (1.0 / 120.0);
        }
    }
    // sum over the B lanes by halving: at offset o each lane keeps the half
    // of its values its bit o selects and adds the partner's copy of it, so
    // lane k ends with the totals of entries k L, ..., k L + L - 1 (L = 16 / B)
    double e[16];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        e[c] = Q[c];
        e[8 + c] = R[c];
    }
    halve_all<B, B / 2>(e, k);
    if (!valid) return;
    constexpr int L = 16 / B;
    const auto bq = rsrc(QR, 16u * Nv * 8u);
#pragma unroll
    for (int i = 0; i < L; ++i) {
        const uint32_t o = ((k * L + i) * Nv + v) * 8u;   // entry-major [16][Nv]
        bstore<double>(bq, o, first ? e[i] : bload<double>(bq, o) + e[i]);
    }
}

// a1[row] = -sum of QR[c][v], a2[row] = -sum of QR[8 + c][v] over the voxels v
// in which the row is corner c, + sum_k phi_k,row t_k,row (as k_gadj_gather)
__global__ __launch_bounds__(kThreads) void k_gadj_vgather(int64_t N, Lattice lat, const double* __restrict__ QR,
                                                           const double* __restrict__ phi, int n_pad, int n_ill,
                                                           int tmode, const double* __restrict__ t_ext,
                                                           const double* __restrict__ W, const double* __restrict__ U,
                                                           double* __restrict__ a1, double* __restrict__ a2) {
    // kSplit (8) lanes per row: lane c takes the voxel in which the row is
    // corner c and the illuminations c, c + 8, ... of the phi t term
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t row = t / kSplit;
    const int c = static_cast<int>(t % kSplit);
    const bool valid = row < N;   // whole groups of kSplit lanes
    const int64_t nx = lat.nx, ny = lat.ny, Nv = (nx - 1) * (ny - 1) * (lat.nz - 1);
    double s1 = 0.0, s2 = 0.0;
    if (valid) {
        const int rx = static_cast<int>(row % nx), ry = static_cast<int>((row / nx) % ny),
                  rz = static_cast<int>(row / (nx * ny));
        const int vx = rx - (c & 1), vy = ry - ((c >> 1) & 1), vz = rz - (c >> 2);
        if (vx >= 0 && vx < nx - 1 && vy >= 0 && vy < ny - 1 && vz >= 0 && vz < lat.nz - 1) {
            const int64_t v = vx + (nx - 1) * (vy + (ny - 1) * (int64_t)vz);
            s1 = -QR[c * Nv + v];
            s2 = -QR[(8 + c) * Nv + v];
        }
        for (int kk = c; kk < n_ill; kk += kSplit) {
            const double tv = tmode == 0 ? t_ext[(int64_t)kk * N + row] : W[row * n_pad + kk] * U[row * n_pad + kk];
            s2 += phi[row * n_pad + kk] * tv;
        }
    }
#pragma unroll
    for (int off = kSplit / 2; off >= 1; off >>= 1) {
        s1 += __shfl_xor(s1, off);
        s2 += __shfl_xor(s2, off);
    }
    if (valid && c == 0) {
        a1[row] = s1;
        a2[row] = s2;
    }
}

// pseudo-random values in [-1, 1) from the index (set-up checks)
__global__ void k_fill_hash(int64_t n, uint64_t seed, double* __restrict__ x) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t h = (static_cast<uint64_t>(i) + seed) * 0x9E3779B97F4A7C15ull;   // splitmix64 finaliser
    h = (h ^ (h >> 30)) * 0xBF58476D1CE4E5B9ull;
    h = (h ^ (h >> 27)) * 0x94D049BB133111EBull;
    h ^= h >> 31;
    x[i] = static_cast<double>(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// out[0] = max |a - b| and out[1] = max |b| as the bits of non-negative doubles
__global__ void k_maxdiff(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                          unsigned long long* out) {
    double d = 0.0, m = 0.0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double e = fabs(a[i] - b[i]);
        if (!(e <= d)) d = e == e ? e : HUGE_VAL;   // a NaN on either side counts as infinite
        m = fmax(m, fabs(b[i]));
    }
    atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(d)));
    atomicMax(out + 1, static_cast<unsigned long long>(__double_as_longlong(m)));
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

inline GeoRef geo_ref(const qpat_ctx* c) { return GeoRef{c->geo, c->geo_cls, c->geo_tab}; }

static VoxGeo vox_geo(const qpat_ctx* c) {
    VoxGeo g;
    for (int d = 0; d < 3; ++d) g.w[d] = 1.0 / (c->vox_h[d] * c->vox_h[d]);
    g.vol = c->vox_h[0] * c->vox_h[1] * c->vox_h[2] / 6.0;
    return g;
}

// k_gadj_vox: 8 equal parts of the voxels (one per XCD), B lanes per voxel
inline dim3 vox_grid(int64_t Nv, int B) {
    const int64_t per_xcd = (Nv + 7) / 8;
    return dim3(static_cast<unsigned>(8 * ((per_xcd * B + kThreads - 1) / kThreads)));
}

// max |a - b| / max |b| over n values (host-synchronous; set-up only)
static qpat_status rel_maxdiff(qpat_ctx* c, int64_t n, const double* a, const double* b, double* rel) {
    unsigned long long* d = nullptr;
    QPAT_TRY(dalloc(c, &d, 2));
    QPAT_HIP(c, hipMemsetAsync(d, 0, 2 * sizeof(unsigned long long), c->stream));
    hipLaunchKernelGGL(k_maxdiff, dim3(grid_for(n, kThreads, 2048)), dim3(kThreads), 0, c->stream, n, a, b, d);
    unsigned long long h[2];
    QPAT_HIP(c, hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    QPAT_TRY(dfree(c, d));
    double dd, mm;
    std::memcpy(&dd, &h[0], sizeof dd);
    std::memcpy(&mm, &h[1], sizeof mm);
    *rel = mm > 0.0 ? dd / mm : (dd > 0.0 ? HUGE_VAL : 0.0);
    return QPAT_OK;
}

// The voxel form assumes Kuhn elements in equal voxels; the lattice check
// only saw the node-node pattern. Before its first use it is compared with
// the element form (any mesh) on pseudo-random coefficients and fields: dK(s)
// rows and the J^T t node sums must agree to 1e-12 relative, else the
// element form stays in use.
static qpat_status vox_check(qpat_ctx* c) {
    if (c->vox != 0) return QPAT_OK;
    c->vox = -1;
    if (!c->lat.on || c->lat.m != 7 || c->opts.operator_format != 1) return QPAT_OK;
    for (int m = 1; m < 8; ++m)   // upper offset with axis mask m in slot m (the Kuhn pattern's order)
        if (c->lat.code[13 + (m & 1) + 3 * ((m >> 1) & 1) + 9 * (m >> 2)] != m) return QPAT_OK;
    const int64_t N = c->N, nx = c->lat.nx, ny = c->lat.ny, nz = c->lat.nz;
    const int64_t Nv = (nx - 1) * (ny - 1) * (nz - 1);
    if (Nv < 1 || 6 * Nv != c->E) return QPAT_OK;
    // the adjoint kernel's 32-bit byte offsets: phi [N][n_pad], blocks [N][16], sums [16][Nv]
    const int64_t lim = (int64_t(1) << 31) - 1;
    if (N * std::max<int64_t>(c->n_pad, 16) * 8 > lim || 16 * Nv * 8 > lim) return QPAT_OK;
    const VoxGeo vg = vox_geo(c);
    const dim3 blk(kThreads);
    constexpr int BC = 16;   // right-hand sides of the check
    double *uu = nullptr, *ue = nullptr, *uv = nullptr, *f = nullptr, *z = nullptr, *tq = nullptr, *tr = nullptr,
           *qr = nullptr, *a = nullptr;
    QPAT_TRY(dalloc(c, &uu, 2 * N));
    QPAT_TRY(dalloc(c, &ue, 8 * N));
    QPAT_TRY(dalloc(c, &uv, 8 * N));
    hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(2 * N, kThreads, 1 << 30)), blk, 0, c->stream, 2 * N, 1ull, uu);
    const dim3 gd((std::min<int64_t>((N * kSplit + kThreads - 1) / kThreads, 4096) + 7) & ~7);
    hipLaunchKernelGGL(k_dk_lattice<8>, gd, blk, 0, c->stream, N, c->lat, c->tets, geo_ref(c), c->n2t_ptr, c->n2t, uu,
                       ue);
    const dim3 gv((std::min<int64_t>((N + kThreads - 1) / kThreads, 4096) + 7) & ~7);
    hipLaunchKernelGGL(k_dk_voxel, gv, blk, 0, c->stream, N, c->lat, vg, uu, uv);
    double rel_dk = 0.0;
    QPAT_TRY(rel_maxdiff(c, 8 * N, uv, ue, &rel_dk));
    QPAT_TRY(dfree(c, uu));
    QPAT_TRY(dfree(c, ue));
    QPAT_TRY(dfree(c, uv));
    if (!(rel_dk <= 1e-12)) return QPAT_OK;
    QPAT_TRY(dalloc(c, &f, BC * N));
    QPAT_TRY(dalloc(c, &z, BC * N));
    QPAT_TRY(dalloc(c, &tq, c->E));
    QPAT_TRY(dalloc(c, &tr, 4 * c->E));
    QPAT_TRY(dalloc(c, &qr, 16 * Nv));
    QPAT_TRY(dalloc(c, &a, 4 * N));
    hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(BC * N, kThreads, 1 << 30)), blk, 0, c->stream, BC * N, 2ull, f);
    hipLaunchKernelGGL(k_fill_hash, dim3(grid_for(BC * N, kThreads, 1 << 30)), blk, 0, c->stream, BC * N, 3ull, z);
    hipLaunchKernelGGL(k_gadj_tet<BC>, dim3(grid_for(c->E * (BC / kTetRhs<BC>), kThreads, 1 << 30)), blk, 0, c->stream,
                       c->E, c->tets, geo_ref(c), f, BC, 0, z, 1, tq, tr);
    hipLaunchKernelGGL(k_gadj_gather, dim3(grid_for(N * kSplit, kThreads, 1 << 30)), blk, 0, c->stream, N, c->n2t_ptr,
                       c->n2t, tq, tr, f, BC, 0, 0, static_cast<const double*>(nullptr),
                       static_cast<const double*>(nullptr), static_cast<const double*>(nullptr), a, a + N);
    hipLaunchKernelGGL(k_gadj_vox<BC>, vox_grid(Nv, BC), blk, 0, c->stream, c->lat, vg, f, BC, 0, z, 1, qr);
    hipLaunchKernelGGL(k_gadj_vgather, dim3(grid_for(N * kSplit, kThreads, 1 << 30)), blk, 0, c->stream, N, c->lat, qr, f, BC, 0,
                       0, static_cast<const double*>(nullptr), static_cast<const double*>(nullptr),
                       static_cast<const double*>(nullptr), a + 2 * N, a + 3 * N);
    double rel1 = 0.0, rel2 = 0.0;
    QPAT_TRY(rel_maxdiff(c, N, a + 2 * N, a, &rel1));
    QPAT_TRY(rel_maxdiff(c, N, a + 3 * N, a + N, &rel2));
    for (double* p : {f, z, tq, tr, qr, a}) QPAT_TRY(dfree(c, p));
    if (rel1 <= 1e-12 && rel2 <= 1e-12) c->vox = 1;
    return QPAT_OK;
}

// K x = b for one block of B right-hand sides: multigrid-preconditioned PCG
// where its hierarchy is built, Jacobi-PCG otherwise

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
        QPAT_TRY(vox_check(c));
        if (c->vox == 1)
            hipLaunchKernelGGL(k_dk_voxel, dim3((std::min<int64_t>((c->N + kThreads - 1) / kThreads, 4096) + 7) & ~7),
                               blk, 0, c->stream, c->N, c->lat, vox_geo(c), c->dKc, c->dK);
        else if (c->lat.m == 7)
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
    QPAT_TRY(vox_check(c));
    const bool vox = c->vox == 1;   // per-voxel sums [Nv][16] in tr (4 E = 24 Nv values)
    const int64_t Nv = vox ? c->E / 6 : 0;
    for (int col0 = 0; col0 < c->n_pad; col0 += B) {
        QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_adj_rhs<BB>, g, blk, 0, c->stream, c->N, c->mu, c->n_pad, c->n_ill,
                                              col0, tmode, t, c->lw, c->lu, c->b64));
        QPAT_TRY(k_solve(c, B, st));
        if (vox) {
            QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_gadj_vox<BB>, vox_grid(Nv, BB), blk, 0, c->stream, c->lat,
                                                  vox_geo(c), c->phi, c->n_pad, col0, c->x64, col0 == 0 ? 1 : 0,
                                                  c->tr));
        } else {
            QPAT_DISPATCH_B(B, hipLaunchKernelGGL(k_gadj_tet<BB>,
                                                  dim3(grid_for(c->E * (BB / kTetRhs<BB>), kThreads, 1 << 30)), blk, 0,
                                                  c->stream, c->E, c->tets, geo_ref(c), c->phi, c->n_pad, col0, c->x64,
                                                  col0 == 0 ? 1 : 0, c->tq, c->tr));
        }
    }
    if (vox)
        hipLaunchKernelGGL(k_gadj_vgather, dim3(grid_for(c->N * kSplit, kThreads, 1 << 30)), blk, 0, c->stream, c->N, c->lat,
                           c->tr, c->phi, c->n_pad, c->n_ill, tmode, t, c->lw, c->lu, c->acc1, c->acc2);
    else
        hipLaunchKernelGGL(k_gadj_gather, dim3(grid_for(c->N * kSplit, kThreads, 1 << 30)), blk, 0, c->stream, c->N,
                           c->n2t_ptr, c->n2t, c->tq, c->tr, c->phi, c->n_pad, c->n_ill, tmode, t, c->lw, c->lu, c->acc1,
                           c->acc2);
    hipLaunchKernelGGL(k_vjp_out, dim3(grid_for(c->N, kThreads, 1 << 30)), blk, 0, c->stream, c->N, c->kappa, c->mu,
                       c->acc1, c->acc2, out, mode == 2 ? 1 : 0, c->lwh, c->ls);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

}  // namespace qpat
