// Geometric multigrid preconditioner for the K and M_delta solves on lattice
// meshes.
//
// K (the forward and adjoint diffusion operator, Sec. 2 and the Appendix) and
// each block of M_delta (Sec. 4 eqs. (4.5), (4.8)) are SPD FEM matrices on the
// node lattice. Their solves are PCG preconditioned by one symmetric V-cycle:
//   * levels: the lattice and its vertex-centred coarsenings, n -> n/2 + 1 per
//     axis, down to the first coarse level of at most kMgDenseK nodes (or at
//     most kMgCoarse nodes per axis);
//   * prolongation P: trilinear interpolation (weights 1, 1/2 per axis),
//     restriction P^T;
//   * coarse operators by Galerkin products A_c = P^T A P, stored like the fine
//     stencil form (diagonal + upper offsets, node-major), 27-point;
//   * smoother: kMgNu weighted Jacobi sweeps before and after the coarse
//     correction, weight 8/(5 g) with g >= lambda_max(D^{-1} A) the Gershgorin
//     bound: the first-degree Chebyshev weight for the interval [g/4, g] that
//     the sweep has to damp; 19/(10 g) on the coarse levels (w lambda < 2
//     keeps the cycle SPD);
//   * coarsest level: the explicit inverse (dense; on the host up to order
//     kMgHostDense, on the GPU above).
// Vectors hold B right-hand sides interleaved ([sys][N][B]); every lane
// (system, right-hand side) has its own PCG scalars and stops on its own.
// With deflation (M_delta: the exact eigenpair (delta, 1) of each block) the
// solve runs on the complement of the constants as the Jacobi-PCG path does:
// b <- b - mean(b), z <- V(r) - mean(V(r)), and the mean of the solution is
// mean(b)/delta. The stopping rule is the same as Jacobi-PCG's:
// ||b - A x||_2 <= rtol ||b||_2 on the FP64 residual, confirmed on the true
// residual at the end. Everything is FP64.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>


#include "qpat_internal.h"

namespace qpat {

struct MgLevel {
    int32_t nx = 0, ny = 0, nz = 0;
    int64_t N = 0;
    int32_t m = 0;                 // stored upper offsets
    int32_t kind = 0;              // row kernel: 0 generic table, 1 Kuhn offsets, 2 27-point, 3 Kuhn upper rows
                                   // entry-major (Uf), 4 whole 27-point rows (Uf)
    const int4* tab = nullptr;     // [m]: dx, dy, dz, dx + nx (dy + ny dz)
    int4* tab_own = nullptr;
    double* U = nullptr;           // [nsys][N][m+1] (level 0: the context's stencil arrays)
    double* dinv = nullptr;        // [nsys][N] 1 / a_ii
    double* b = nullptr;           // [nsys][N][B] (level 0: the PCG residual)
    double* x = nullptr;           // [nsys][N][B]
    double* t = nullptr;           // ping-pong partner of x
    double* r = nullptr;           // residual before restriction
    double* W = nullptr;           // [nsys][8][N] operator-dependent prolongation weights to the next level (corner-major)
    float* Wc = nullptr;           // [nsys][WPack size] the nonzero ones of W in FP32, packed by corner: the V-cycle's
                                   // transfers read these (W holds the same rounded values for the Galerkin set-up:
                                   // one P throughout)
    double* Uf = nullptr;          // kind 3: [nsys][kUpRow][N] Kuhn diagonal + upper entries, entry-major;
                                   // K level 0: [N][kFullRow] whole Kuhn rows; K levels >= 1: [N][kRow27]
    float* Uf32 = nullptr;         // kind 5 / 6: the kind-3 / kind-4 rows in FP32 (M_delta's V-cycle)
    float* Ufk32 = nullptr;        // K level 0: the whole Kuhn rows [N][16] in FP32 (fused prolongation + last sweep)
    float* Uf27p = nullptr;        // K tiled levels >= 1: the 27-point rows in FP32 as [N][16] pairs (entry k, entry k + 16)
    int32_t vkind = -1;            // row kind of the V-cycle's kernels on this level (-1: kind)
};

struct MgScal {
    double rz, pq, alpha, beta, c, rr, bnorm2, mean;
    int32_t active, done, iters, pad;
};

// Tiling of the finest level for one block size (LDS-tiled kernels)
constexpr int kMgMaxLevels = 12;   // levels with a tiled-kernel geometry (more levels run untiled)
struct TileGeo {
    bool ready = false, on = false;
    int32_t tiles_x = 0, tiles_y = 0, zc = 0, items = 0, blocks = 0;
    // the tiled restrictions, level l to l + 1 (coarse tiles, coarse z-chunk, blocks)
    struct Rst {
        bool on = false;
        int32_t tx = 0, ty = 0, zc = 0, items = 0, blocks = 0;
    };
    Rst rst[kMgMaxLevels];
    // the fused prolongation + last sweep (16 right-hand sides; even z-chunks)
    bool ps_on = false;
    int32_t ps_zc = 0, ps_items = 0, ps_blocks = 0;
    int32_t ps_zc32 = 0, ps_items32 = 0, ps_blocks32 = 0;   // its FP32-staged form
    // the cost model's z-chunk lengths (tiles, prolongation + sweep FP64, FP32) and whether
    // the ones in use were picked by timing them (autotune)
    int32_t zc_model = 0, ps_zc_model = 0, ps_zc32_model = 0;
    bool tuned = false;
    // the tiled 27-point kernels of the coarse levels (16 right-hand sides)
    struct Lv27 {
        bool on = false;
        int32_t tx = 0, ty = 0, zc = 0, items = 0, blocks = 0;
    };
    Lv27 t27[kMgMaxLevels];
};

struct MgState {
    int32_t nsys = 1;              // 1 (K) or 2 (the blocks of M_delta)
    bool opdep = false;            // operator-dependent prolongation (else trilinear)
    int32_t bmax = 1;              // right-hand sides the vectors are sized for
    bool current = false;          // built from the operator now assembled
    std::vector<MgLevel> lv;
    double* w = nullptr;           // [nsys][levels] Jacobi weights
    double* ainv = nullptr;        // [nsys][Nc][Nc]
    double *pr = nullptr, *pa = nullptr, *pb = nullptr, *pq = nullptr;  // PCG r, p (two), q: [nsys][N][bmax]
    double* pr2 = nullptr;         // the other residual buffer of the fused update (odd iterations write r here)
    double* pring = nullptr;       // [kRing][N][bmax] directions of the tiled iterations (FP32 or FP64 elements)
    double* ahist = nullptr;       // [kRing][lanes] their alphas (0: the lane did not iterate)
    int32_t* pslot = nullptr;      // iterations of the current run so far (the ring slot of the next one)
    double* parts = nullptr;       // [lanes][4][kMgBlocks]
    uint64_t* gmax = nullptr;      // [nsys][levels] Gershgorin bounds (bit patterns)
    MgScal* sc = nullptr;          // [lanes], lane = sys B + k
    MgScal* sc_host = nullptr;
    // region coarse space (M_delta): z += Z E^{-1} Z^T r, E = Z^T A Z
    int32_t kreg = 0;              // regions of the system with most (0: off)
    int32_t nreg[2] = {0, 0};
    int32_t* reg = nullptr;        // [nsys][N] region of each node, -1: none
    double* einv = nullptr;        // [nsys][kRegMax][kRegMax]
    double* rsize = nullptr;       // [nsys][kRegMax] nodes per region
    double* rparts = nullptr;      // [nsys][kRegMax][kMgBlocks] partial sums of Z^T r
    double* ry = nullptr;          // [nsys][kRegMax] y = E^{-1} Z^T r
    double* rcorr = nullptr;       // [nsys][2] r.(Z y), mean(Z y) (0 without deflation)
    std::map<int, TileGeo> tiles;  // by block size
    std::vector<hipEvent_t> ev;    // per-launch timing (profiling)
    std::map<std::string, hipGraphExec_t> graphs;
    hipStream_t cap = nullptr;
};

namespace {

constexpr int kMgCoarse = 5;      // coarsest lattice: at most this many nodes per axis, or
constexpr int64_t kMgDenseK = 1000;   // the first coarse level of at most this many nodes
constexpr int64_t kMgHostDense = 256;   // coarsest inverses up to this order on the host, larger ones on the GPU
constexpr int kMgNu = 1;          // Jacobi sweeps before and after the coarse correction
constexpr int kMgBlocks = 2048;   // most blocks of a kernel that writes partial sums (8 per CU)
constexpr int kMgGrid = 512;      // blocks of the vector kernels of several right-hand sides
constexpr int kMgT = 256;
constexpr int kMgLanes = 32;      // systems x right-hand sides
constexpr int kMgChunk0 = 4;      // PCG iterations before the first host check of a run
// The tiled K iterations keep their last kRing directions and alphas instead of
// updating x each iteration; x is formed from them before it is read (the
// true residual) or when the ring is full.
constexpr int kRing = 16;
// Region coarse space of M_delta: regions are the connected components of the
// graph of strong couplings |a_ij| > kRegTheta sqrt(a_ii a_jj); the kRegMax
// largest with at least kRegMin nodes get an indicator vector.
constexpr int kRegMax = 16;
constexpr int kRegMin = 64;
constexpr double kRegTheta = 1e-2;
constexpr int kRegList = 4096;    // candidate regions collected per system

__device__ __forceinline__ void coords(int32_t i, int nx, int ny, int& ix, int& iy, int& iz) {
    ix = i % nx;
    const int32_t q = i / nx;
    iy = q % ny;
    iz = q / ny;
}

// (A x)_i of lane k (x interleaved [N][B]), and sum_j |a_ij| when ABS
template <bool ABS, int B>
__device__ __forceinline__ double st_row(const double* __restrict__ U, int M1, const int4* __restrict__ tab, int m,
                                         int nx, int ny, int nz, const double* __restrict__ x, int32_t i, int k) {
    int ix, iy, iz;
    coords(i, nx, ny, ix, iy, iz);
    double s = ABS ? fabs(U[(int64_t)i * M1]) : U[(int64_t)i * M1] * x[(int64_t)i * B + k];
    for (int j = 0; j < m; ++j) {
        const int4 t = tab[j];
        const int ux = ix + t.x, uy = iy + t.y, uz = iz + t.z;
        if (ux >= 0 && ux < nx && uy >= 0 && uy < ny && uz < nz) {
            const double a = U[(int64_t)i * M1 + j + 1];
            s += ABS ? fabs(a) : a * x[(int64_t)(i + t.w) * B + k];
        }
        const int lx = ix - t.x, ly = iy - t.y, lz = iz - t.z;
        if (lx >= 0 && lx < nx && ly >= 0 && ly < ny && lz >= 0) {
            const double a = U[(int64_t)(i - t.w) * M1 + j + 1];
            s += ABS ? fabs(a) : a * x[(int64_t)(i - t.w) * B + k];
        }
    }
    return s;
}
// The rows with compile-time offsets: KIND 1 the Kuhn split (7 upper offsets,
// the fine level of a Kuhn mesh), KIND 2 the full 27-point stencil (13 upper
// offsets in code order, the Galerkin levels); KIND 0 the generic table.
constexpr int kKx[7] = {1, 0, 1, 0, 1, 0, 1};
constexpr int kKy[7] = {0, 1, 1, 0, 0, 1, 1};
constexpr int kKz[7] = {0, 0, 0, 1, 1, 1, 1};

// The stencil and V-cycle kernels give each thread V = 2 adjacent right-hand
// sides of one node (16-byte loads and stores; the row of the operator is read
// once for both); BV = B / V threads share a node.
typedef double d2v __attribute__((ext_vector_type(2)));
template <int B>
struct Pk {
    static constexpr int V = B >= 2 ? 2 : 1;
    static constexpr int BV = B / V;
};
template <int V>
struct VecT {
    using T = double;
};
template <>
struct VecT<2> {
    using T = d2v;
};
template <int B>
using TB = typename VecT<Pk<B>::V>::T;

template <typename T>
__device__ __forceinline__ T vld(const double* p) {
    return *reinterpret_cast<const T*>(p);
}
template <typename T>
__device__ __forceinline__ void vst(double* p, T v) {
    *reinterpret_cast<T*>(p) = v;
}
// the same from / to FP32 storage (a coarse level's vectors kept in FP32)
template <typename T>
__device__ __forceinline__ T vldf(const float* p) {
    if constexpr (sizeof(T) == 8) {
        return static_cast<double>(*p);
    } else {
        typedef float f2v __attribute__((ext_vector_type(2)));
        const f2v t = *reinterpret_cast<const f2v*>(p);
        return T{static_cast<double>(t.x), static_cast<double>(t.y)};
    }
}
template <typename T>
__device__ __forceinline__ void vstf(float* p, T v) {
    if constexpr (sizeof(T) == 8) {
        *p = static_cast<float>(v);
    } else {
        typedef float f2v __attribute__((ext_vector_type(2)));
        *reinterpret_cast<f2v*>(p) = f2v{static_cast<float>(v.x), static_cast<float>(v.y)};
    }
}
// vectors kept in FP64 or in FP32, by the pointer's type
template <typename T>
__device__ __forceinline__ T vldx(const double* p) {
    return vld<T>(p);
}
template <typename T>
__device__ __forceinline__ T vldx(const float* p) {
    return vldf<T>(p);
}
template <typename T>
__device__ __forceinline__ void vstx(double* p, T v) {
    vst<T>(p, v);
}
template <typename T>
__device__ __forceinline__ void vstx(float* p, T v) {
    vstf<T>(p, v);
}
// v as a vector of element type VT holds it (FP32: rounded)
template <typename VT>
__device__ __forceinline__ double held_as(double v) {
    return static_cast<double>(static_cast<VT>(v));
}
__device__ __forceinline__ double comp(double v, int) { return v; }
__device__ __forceinline__ double comp(d2v v, int c) { return c ? v.y : v.x; }

// Node order of the stencil kernels. The blocks of XCD x (block b runs on XCD
// b mod 8) take the y-strip [x ny / 8, (x + 1) ny / 8) of every plane (z-slabs
// when ny < 8) and sweep it plane by plane, x fastest. The strip's planes
// around the sweep (about 0.3 MB per plane of a 129^2 lattice with 16
// right-hand sides) then stay in that XCD's 4 MB L2 while the up to 27
// neighbours of every node are read, so each vector comes from HBM about
// once. Calls f(ix, iy, iz, node, thread-in-node). The thread-in-node is
// threadIdx.x mod BV for every element of a thread.
template <int BV, typename F>
__device__ __forceinline__ void walk(int32_t nx, int32_t ny, int32_t nz, F&& f) {
    const int32_t xcd = blockIdx.x & 7;
    int32_t y0 = 0, ys = ny, z0 = 0, zs = nz;
    if (ny >= 8) {
        y0 = xcd * ny / 8;
        ys = (xcd + 1) * ny / 8 - y0;
    } else {
        z0 = xcd * nz / 8;
        zs = (xcd + 1) * nz / 8 - z0;
    }
    const int32_t total = nx * ys * zs * BV;
    const int32_t step = (gridDim.x >> 3) * kMgT;
    for (int32_t e = (blockIdx.x >> 3) * kMgT + threadIdx.x; e < total; e += step) {
        const int32_t v = e % BV, n = e / BV;
        const int32_t ix = n % nx, q = n / nx;
        const int32_t iy = y0 + q % ys, iz = z0 + q / ys;
        f(ix, iy, iz, ix + nx * (iy + ny * iz), v);
    }
}

struct LvArgs {
    const double* U;
    const int4* tab;
    int32_t m, nx, ny, nz;
    int64_t N;
    int32_t kind;         // row kernel: 0 generic table, 1 Kuhn offsets, 2 full 27-point, 3 Kuhn upper rows
                          // entry-major, 4 27-point whole rows entry-major (5, 6: 3, 4 in FP32)
    const double* Uf;     // kind 3: [nsys][kUpRow][N]; kind 4: [nsys][27][N]
    const float* Uf32;    // kind 5 / 6: the same in FP32
};

// Kuhn rows for the one-right-hand-side kernels: the diagonal and the 7 upper
// entries, entry-major ([kUpRow][N] per system), so that a wavefront's loads of
// one entry for consecutive nodes are contiguous, the lower entries included
// (each is a partner row's upper entry at a shifted index)
constexpr int kUpRow = 8;
// whole Kuhn rows (diagonal, 7 upper, 7 lower entries, pad), node-major, for
// the 16-lane fused prolongation + sweep
constexpr int kFullRow = 16;

// first stored row of system sys in the form the row kernel KIND reads
template <int KIND>
__device__ __forceinline__ const double* rows_of(const LvArgs& L, int sys) {
    if constexpr (KIND == 3) return L.Uf + (int64_t)sys * L.N * kUpRow;
    if constexpr (KIND == 4) return L.Uf + (int64_t)sys * L.N * 27;
    if constexpr (KIND == 6) return reinterpret_cast<const double*>(L.Uf32 + (int64_t)sys * L.N * 27);
    if constexpr (KIND == 5) return reinterpret_cast<const double*>(L.Uf32 + (int64_t)sys * L.N * kUpRow);
    return L.U + (int64_t)sys * L.N * (L.m + 1);
}

// (A x)_i for the thread's V right-hand sides; x points at the thread's
// first right-hand side of node 0 ([N][B] interleaved). Interior rows skip
// the lattice-edge tests.
template <int KIND, int B, typename XT = double>
__device__ __forceinline__ TB<B> apply(const LvArgs& L, const double* __restrict__ U, const XT* __restrict__ x,
                                       int32_t ix, int32_t iy, int32_t iz, int32_t i) {
    using T = TB<B>;
    if constexpr (KIND == 0) {
        const int32_t M1 = L.m + 1;
        T s = U[i * M1] * vldx<T>(x + i * B);
        for (int j = 0; j < L.m; ++j) {
            const int4 t = L.tab[j];
            if (ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz)
                s += U[i * M1 + j + 1] * vldx<T>(x + (i + t.w) * B);
            if (ix - t.x >= 0 && ix - t.x < L.nx && iy - t.y >= 0 && iy - t.y < L.ny && iz - t.z >= 0)
                s += U[(i - t.w) * M1 + j + 1] * vldx<T>(x + (i - t.w) * B);
        }
        return s;
    } else if constexpr (KIND == 4) {   // 27-point whole rows, entry-major ([27][N])
        const bool inner = ix > 0 && ix < L.nx - 1 && iy > 0 && iy < L.ny - 1 && iz > 0 && iz < L.nz - 1;
        T s = U[i] * vldx<T>(x + i * B);
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            const int code = 14 + j;
            const int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
            const int32_t lin = dx + L.nx * (dy + L.ny * dz);
            const bool up = inner || (ix + dx >= 0 && ix + dx < L.nx && iy + dy >= 0 && iy + dy < L.ny && iz + dz < L.nz);
            const bool lo = inner || (ix - dx >= 0 && ix - dx < L.nx && iy - dy >= 0 && iy - dy < L.ny && iz - dz >= 0);
            // loads from clamped indices and selected sums: no branch per
            // neighbour, so all of a row's loads are in flight together
            const T xu = vldx<T>(x + (up ? i + lin : i) * B), xl = vldx<T>(x + (lo ? i - lin : i) * B);
            const double cu = U[(1 + j) * L.N + i], cl = U[(14 + j) * L.N + i];
            s = up ? s + cu * xu : s;
            s = lo ? s + cl * xl : s;
        }
        return s;
    } else if constexpr (KIND == 6) {   // the kind-4 rows in FP32 (a preconditioner's coarse operator)
        const float* Uw = reinterpret_cast<const float*>(U);
        const bool inner = ix > 0 && ix < L.nx - 1 && iy > 0 && iy < L.ny - 1 && iz > 0 && iz < L.nz - 1;
        T s = static_cast<double>(Uw[i]) * vldx<T>(x + i * B);
#pragma unroll
        for (int j = 0; j < 13; ++j) {
            const int code = 14 + j;
            const int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
            const int32_t lin = dx + L.nx * (dy + L.ny * dz);
            const bool up = inner || (ix + dx >= 0 && ix + dx < L.nx && iy + dy >= 0 && iy + dy < L.ny && iz + dz < L.nz);
            const bool lo = inner || (ix - dx >= 0 && ix - dx < L.nx && iy - dy >= 0 && iy - dy < L.ny && iz - dz >= 0);
            const T xu = vldx<T>(x + (up ? i + lin : i) * B), xl = vldx<T>(x + (lo ? i - lin : i) * B);
            const double cu = static_cast<double>(Uw[(1 + j) * L.N + i]), cl = static_cast<double>(Uw[(14 + j) * L.N + i]);
            s = up ? s + cu * xu : s;
            s = lo ? s + cl * xl : s;
        }
        return s;
    } else if constexpr (KIND == 3 || KIND == 5) {
        // Kuhn rows' diagonal and upper entries, entry-major (3: FP64, 5: FP32).
        // The lower entry of offset j of row i is the upper entry j of row
        // i - u_j, read at the shifted index of the same entry array: the
        // partner row's entries were read moments before in the sweep order,
        // so the shifted reads come from L2 and each row crosses HBM once.
        using W = std::conditional_t<KIND == 5, float, double>;
        const W* Uw = reinterpret_cast<const W*>(U);
        double u[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) u[k] = static_cast<double>(Uw[k * L.N + i]);
        const bool inner = ix > 0 && ix < L.nx - 1 && iy > 0 && iy < L.ny - 1 && iz > 0 && iz < L.nz - 1;
        T s = u[0] * vldx<T>(x + i * B);
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const int dx = kKx[j], dy = kKy[j], dz = kKz[j];
            const int32_t lin = dx + L.nx * (dy + L.ny * dz);
            const bool up = inner || (ix + dx < L.nx && iy + dy < L.ny && iz + dz < L.nz);
            const bool lo = inner || (ix - dx >= 0 && iy - dy >= 0 && iz - dz >= 0);
            const int32_t il = lo ? i - lin : i;
            const T xu = vldx<T>(x + (up ? i + lin : i) * B), xl = vldx<T>(x + il * B);
            const double cl = static_cast<double>(Uw[(1 + j) * L.N + il]);
            s = up ? s + u[1 + j] * xu : s;
            s = lo ? s + cl * xl : s;
        }
        return s;
    } else {
        constexpr int MM = KIND == 1 ? 7 : 13;
        constexpr int M1 = MM + 1;   // even: the row is M1 / 2 16-byte loads
        double u[M1];
        const d2v* Ur = reinterpret_cast<const d2v*>(U + i * M1);
#pragma unroll
        for (int k = 0; k < M1 / 2; ++k) {
            const d2v t = Ur[k];
            u[2 * k] = t.x;
            u[2 * k + 1] = t.y;
        }
        const bool inner = ix > 0 && ix < L.nx - 1 && iy > 0 && iy < L.ny - 1 && iz > 0 && iz < L.nz - 1;
        T s = u[0] * vldx<T>(x + i * B);
#pragma unroll
        for (int j = 0; j < MM; ++j) {
            const int code = 14 + j;
            const int dx = KIND == 1 ? kKx[j] : code % 3 - 1;
            const int dy = KIND == 1 ? kKy[j] : (code / 3) % 3 - 1;
            const int dz = KIND == 1 ? kKz[j] : code / 9 - 1;
            const int32_t lin = dx + L.nx * (dy + L.ny * dz);
            const bool up = inner || (ix + dx >= 0 && ix + dx < L.nx && iy + dy >= 0 && iy + dy < L.ny && iz + dz < L.nz);
            const bool lo = inner || (ix - dx >= 0 && ix - dx < L.nx && iy - dy >= 0 && iy - dy < L.ny && iz - dz >= 0);
            const int32_t il = lo ? i - lin : i;
            const T xu = vldx<T>(x + (up ? i + lin : i) * B), xl = vldx<T>(x + il * B);
            const double cl = U[il * M1 + j + 1];
            s = up ? s + u[j + 1] * xu : s;
            s = lo ? s + cl * xl : s;
        }
        return s;
    }
}

// Compensated accumulation of s - a x: the product's rounding error comes
// from a fused multiply-add and the sum's from a two-sum, so that s + c holds
// b - sum a_j x_j to a few ulps of the result instead of ulps of
// sum |a_j x_j| (the true residual near the attainable accuracy of PCG).
struct CompSum {
    double s, c;
    __device__ __forceinline__ explicit CompSum(double b) : s(b), c(0.0) {}
    __device__ __forceinline__ void sub(double a, double x) {
        const double p = a * x;
        const double e = fma(a, x, -p);   // a x = p + e exactly
        const double t = s - p;
        const double bp = t - s;
        const double err = (s - (t - bp)) + (-p - bp);   // s - p = t + err exactly
        s = t;
        c += err - e;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

// b_i - (A x)_i of one right-hand side (x: its entry of node 0, stride B),
// compensated; any stencil form (the offset table)
template <int B>
__device__ double resid_comp(const LvArgs& L, const double* __restrict__ U, const double* __restrict__ x, double bi,
                             int32_t ix, int32_t iy, int32_t iz, int32_t i) {
    const int32_t M1 = L.m + 1;
    CompSum r(bi);
    r.sub(U[i * M1], x[i * B]);
    for (int j = 0; j < L.m; ++j) {
        const int4 t = L.tab[j];
        if (ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz)
            r.sub(U[i * M1 + j + 1], x[(i + t.w) * B]);
        if (ix - t.x >= 0 && ix - t.x < L.nx && iy - t.y >= 0 && iy - t.y < L.ny && iz - t.z >= 0)
            r.sub(U[(i - t.w) * M1 + j + 1], x[(i - t.w) * B]);
    }
    return r.value();
}

// The same for a stencil form of 7 offsets (the Kuhn lattice), all loads in
// flight before the sums: indices clamped to the node itself and the terms of
// neighbours off the lattice replaced by 0 * 0, which the compensated sum
// takes exactly (so the value is bitwise that of resid_comp).
template <int B>
__device__ double resid_comp7(const LvArgs& L, const double* __restrict__ U, const double* __restrict__ x, double bi,
                              int32_t ix, int32_t iy, int32_t iz, int32_t i) {
    constexpr int32_t M1 = 8;
    double cu[7], xu[7], cl[7], xl[7];
    const double c0 = U[i * M1], x0 = x[i * B];
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int4 t = L.tab[j];
        const bool up = ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz;
        const bool lo = ix - t.x >= 0 && ix - t.x < L.nx && iy - t.y >= 0 && iy - t.y < L.ny && iz - t.z >= 0;
        const int32_t iu = up ? i + t.w : i, il = lo ? i - t.w : i;
        const double a = U[i * M1 + j + 1], xa = x[iu * B], c = U[il * M1 + j + 1], xc = x[il * B];
        cu[j] = up ? a : 0.0;
        xu[j] = up ? xa : 0.0;
        cl[j] = lo ? c : 0.0;
        xl[j] = lo ? xc : 0.0;
    }
    CompSum r(bi);
    r.sub(c0, x0);
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        r.sub(cu[j], xu[j]);
        r.sub(cl[j], xl[j]);
    }
    return r.value();
}

// plain grid-stride loop over n elements (one right-hand side each; the lane
// of a thread is threadIdx.x mod B)
#define QPAT_MG_ELEMS(e, n) \
    for (int64_t e = blockIdx.x * (int64_t)kMgT + threadIdx.x; e < (n); e += (int64_t)gridDim.x * kMgT)

// Sum over the threads with equal threadIdx.x mod G; the result is valid in
// threads threadIdx.x < G (group threadIdx.x).
template <int G>
__device__ __forceinline__ double group_sum(double v, double* sm) {
#pragma unroll
    for (int off = 32; off >= G; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < G) sm[wave * G + lane] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < G)
        for (int w = 0; w < kMgT / 64; ++w) t += sm[w * G + threadIdx.x];
    __syncthreads();
    return t;
}

// any of the V right-hand sides of thread-in-node v of system sys still iterating
template <int B>
__device__ __forceinline__ bool pair_active(const MgScal* sc, int sys, int v) {
    bool on = false;
#pragma unroll
    for (int c = 0; c < Pk<B>::V; ++c) on = on || sc[sys * B + v * Pk<B>::V + c].active;
    return on;
}

// partial sums of the block: parts[lane][slot][block]
// a block's partial sum; a grid smaller than kMgBlocks also clears the slots
// no block of it owns, so that the reductions can read a fixed count
__device__ __forceinline__ void put(double* parts, int lane, int slot, double val) {
    double* p = parts + (lane * 4 + slot) * kMgBlocks;
    p[blockIdx.x] = val;
    for (int b = blockIdx.x + gridDim.x; b < kMgBlocks; b += gridDim.x) p[b] = 0.0;
}

// per-right-hand-side block sums of a V-wide accumulator, written as partials
template <int B>
__device__ __forceinline__ void put_sums(double* parts, int sys, int slot, TB<B> acc, double* sm) {
#pragma unroll
    for (int c = 0; c < Pk<B>::V; ++c) {
        const double t = group_sum<Pk<B>::BV>(comp(acc, c), sm);
        if (threadIdx.x < Pk<B>::BV) put(parts, sys * B + threadIdx.x * Pk<B>::V + c, slot, t);
    }
}

// Kuhn rows from the stencil form (zero where the partner is off the lattice):
// ENTRY, the row kind 3, the diagonal and upper entries entry-major
// [kUpRow][N]; otherwise whole rows node-major [N][kFullRow] (the lower entries
// gathered from the partner rows) for the 16-lane kernels
template <bool ENTRY>
__global__ __launch_bounds__(kMgT) void k_mg_fullrows(LvArgs L, double* __restrict__ Uf) {
    const int sys = blockIdx.y;
    constexpr int M1 = 8;
    const double* U = L.U + (int64_t)sys * L.N * M1;
    double* F = Uf + (int64_t)sys * L.N * (ENTRY ? kUpRow : kFullRow);
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        double u[kFullRow];
        u[0] = U[i * M1];
#pragma unroll
        for (int j = 0; j < 7; ++j) {
            const int dx = kKx[j], dy = kKy[j], dz = kKz[j];
            const int64_t lin = dx + (int64_t)L.nx * (dy + (int64_t)L.ny * dz);
            const bool up = ix + dx < L.nx && iy + dy < L.ny && iz + dz < L.nz;
            const bool lo = ix - dx >= 0 && iy - dy >= 0 && iz - dz >= 0;
            u[1 + j] = up ? U[i * M1 + 1 + j] : 0.0;
            u[8 + j] = lo ? U[(i - lin) * M1 + 1 + j] : 0.0;
        }
        u[15] = 0.0;
        if constexpr (ENTRY) {
#pragma unroll
            for (int k = 0; k < kUpRow; ++k) F[k * L.N + i] = u[k];
        } else {
#pragma unroll
            for (int k = 0; k < kFullRow; ++k) F[i * kFullRow + k] = u[k];
        }
    }
}

__global__ __launch_bounds__(kMgT) void k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMgT)
        b[i] = static_cast<float>(a[i]);
}

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
        const double row = st_row<true, 1>(U, M1, L.tab, L.m, L.nx, L.ny, L.nz, nullptr, static_cast<int32_t>(i), 0);
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

// Prolongation weight of fine node i (coords fx, fy, fz) towards coarse node
// J0(i) + corner c, J0(i) = (fx/2, fy/2, fz/2), c = cz 4 + cy 2 + cx. W: the
// operator-dependent weights of the system, corner-major ([8][N]: the loads of
// one corner for consecutive nodes are contiguous), or null for trilinear
// interpolation (1 on an even axis, 1/2 to both sides on an odd one).
__device__ __forceinline__ double pweight(const double* __restrict__ W, int64_t N, int64_t i, int fx, int fy, int fz,
                                          int c) {
    if (W) return W[c * N + i];
    const int bx = c & 1, by = (c >> 1) & 1, bz = c >> 2;
    const double wx = (fx & 1) ? 0.5 : (bx ? 0.0 : 1.0);
    const double wy = (fy & 1) ? 0.5 : (by ? 0.0 : 1.0);
    const double wz = (fz & 1) ? 0.5 : (bz ? 0.0 : 1.0);
    return wx * wy * wz;
}

// Packed prolongation weights. Fine node (ix, iy, iz) takes its value from the
// corners J0 + (a, b, c) of the coarse cell J0 = (ix/2, iy/2, iz/2). Along an
// axis where the node's coordinate is even it lies on a coarse plane, so a
// corner one step up that axis has weight 0 (trilinear and operator-dependent
// alike: the collapsed stencil has no extent along an even axis). Corner
// cn = a + 2 b + 4 c is therefore kept only on the sub-lattice of nodes that are
// odd along every axis of its set bits, indexed (a ? ix/2 : ix, b ? iy/2 : iy,
// c ? iz/2 : iz); the eight sub-lattices follow one another in corner order,
// 27/8 values per node instead of 8.
struct WPack {
    int32_t nx, ny, nz;
    __host__ __device__ __forceinline__ int64_t size() const {
        return (int64_t)(nx + (nx >> 1)) * (ny + (ny >> 1)) * (nz + (nz >> 1));
    }
    // (32-bit: the set-up keeps size() below 2^31)
    __device__ __forceinline__ int32_t at(int cn, int32_t ix, int32_t iy, int32_t iz) const {
        const int a = cn & 1, b = (cn >> 1) & 1, c = cn >> 2;
        const int32_t sx = a ? nx >> 1 : nx, sy = b ? ny >> 1 : ny, sz = c ? nz >> 1 : nz;
        const int32_t off = (c ? (nx + (nx >> 1)) * (ny + (ny >> 1)) * nz : 0) + (b ? (nx + (nx >> 1)) * ny * sz : 0) +
                            (a ? nx * sy * sz : 0);
        return off + (a ? ix >> 1 : ix) + sx * ((b ? iy >> 1 : iy) + sy * (c ? iz >> 1 : iz));
    }
    // at() for any node inside the lattice, clamped into the array: a load that
    // is always in bounds, whose value is used only where held() is true
    __device__ __forceinline__ int32_t atc(int cn, int32_t ix, int32_t iy, int32_t iz) const {
        return min(at(cn, ix, iy, iz), static_cast<int32_t>(size() - 1));
    }
    // whether corner cn can carry a nonzero weight for node (ix, iy, iz)
    __device__ __forceinline__ static bool held(int cn, int32_t ix, int32_t iy, int32_t iz) {
        return !((cn & 1) && !(ix & 1)) && !((cn & 2) && !(iy & 1)) && !((cn & 4) && !(iz & 1));
    }
};

// W rounded to FP32 in place (the Galerkin product then uses exactly the values
// the transfers apply) and its nonzero entries packed into Wc
__global__ __launch_bounds__(kMgT) void k_mg_wpack(LvArgs L, double* __restrict__ Wall, float* __restrict__ Wc) {
    const int sys = blockIdx.y;
    const WPack pk{L.nx, L.ny, L.nz};
    double* W = Wall + (int64_t)sys * L.N * 8;
    float* P = Wc + sys * pk.size();
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        for (int cn = 0; cn < 8; ++cn) {
            const float v = static_cast<float>(W[cn * L.N + i]);
            W[cn * L.N + i] = static_cast<double>(v);
            if (WPack::held(cn, ix, iy, iz)) P[pk.at(cn, ix, iy, iz)] = v;
        }
    }
}

// Galerkin coarse operator A_c = P^T A P, diagonal and the 13 upper offsets
// (code order (dx+1) + 3 (dy+1) + 9 (dz+1) = 13 ... 26) of every coarse node:
// sum over the fine nodes i in the support of I, the fine stencil entries
// a_ij, and the coarse nodes J whose support holds j, of P(i,I) a_ij P(j,J).
// W: [nsys][8][N] weights of P, or null (trilinear).
__global__ __launch_bounds__(kMgT) void k_mg_rap(LvArgs F, const double* __restrict__ Wall, double* __restrict__ Uc,
                                                 int cx, int cy, int cz) {
    __shared__ double acc[kMgT][14];
    const int sys = blockIdx.y;
    const int64_t Nc = (int64_t)cx * cy * cz;
    const int64_t I = blockIdx.x * (int64_t)kMgT + threadIdx.x;
    const int Mf = F.m + 1;
    const double* U = F.U + (int64_t)sys * F.N * Mf;
    const double* W = Wall ? Wall + (int64_t)sys * F.N * 8 : nullptr;
    for (int k = 0; k < 14; ++k) acc[threadIdx.x][k] = 0.0;
    if (I < Nc) {
        int Ix, Iy, Iz;
        coords(static_cast<int32_t>(I), cx, cy, Ix, Iy, Iz);
        for (int di = 0; di < 27; ++di) {
            const int ax = di % 3 - 1, ay = (di / 3) % 3 - 1, az = di / 9 - 1;
            const int fx = 2 * Ix + ax, fy = 2 * Iy + ay, fz = 2 * Iz + az;
            if (fx < 0 || fx >= F.nx || fy < 0 || fy >= F.ny || fz < 0 || fz >= F.nz) continue;
            const int32_t i = fx + F.nx * (fy + F.ny * fz);
            // I = J0(i) + corner, corner 1 exactly along the axes where i sits below 2 I
            const double wi = pweight(W, F.N, i, fx, fy, fz, (ax < 0 ? 1 : 0) + (ay < 0 ? 2 : 0) + (az < 0 ? 4 : 0));
            if (wi == 0.0) continue;
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
                const int32_t j = i + lin;
                for (int cj = 0; cj < 8; ++cj) {
                    const double wj = pweight(W, F.N, j, jx, jy, jz, cj);
                    if (wj == 0.0) continue;
                    const int Jx = (jx >> 1) + (cj & 1), Jy = (jy >> 1) + ((cj >> 1) & 1), Jz = (jz >> 1) + (cj >> 2);
                    const int code = (Jx - Ix + 1) + 3 * (Jy - Iy + 1) + 9 * (Jz - Iz + 1);
                    if (code < 13) continue;   // lower half: stored at the partner row
                    acc[threadIdx.x][code - 13] += wi * a * wj;
                }
            }
        }
        double* out = Uc + ((int64_t)sys * Nc + I) * 14;
        for (int k = 0; k < 14; ++k) out[k] = acc[threadIdx.x][k];
    }
}

// ------------------------------------------------ operator-dependent transfer
// Prolongation weights from the operator (M_delta, whose diffusivity drops by
// orders of magnitude across the edges of the image). A fine node with one odd
// coordinate takes its two coarse neighbours along that axis with weights
// -C(-1)/C(0), -C(+1)/C(0) of its stencil collapsed onto the axis (summed
// over the two even axes); one with two odd coordinates combines its eight
// in-plane neighbours (interpolated already) with the stencil collapsed over
// the even axis; one with three odd coordinates its 26 neighbours with the
// stencil itself. Across an interface the weights towards the weakly coupled
// side vanish, so the coarse levels keep the regions apart where trilinear
// interpolation would mix them. A node whose collapsed centre is not positive,
// or that has no +1 neighbour along an odd axis, keeps the trilinear weights.
// Parity class = number of odd coordinates; classes run in order 0 ... 3.
template <int CLASS>
__global__ __launch_bounds__(kMgT) void k_mg_pweights(LvArgs L, double* __restrict__ Wall) {
    const int sys = blockIdx.y;
    const int M1 = L.m + 1;
    const double* U = L.U + (int64_t)sys * L.N * M1;
    double* W = Wall + (int64_t)sys * L.N * 8;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        const int px = ix & 1, py = iy & 1, pz = iz & 1;
        if (px + py + pz != CLASS) continue;
        double w[8];
        for (int c = 0; c < 8; ++c) w[c] = pweight(nullptr, L.N, i, ix, iy, iz, c);
        bool ok = CLASS > 0 && !(px && ix + 1 >= L.nx) && !(py && iy + 1 >= L.ny) && !(pz && iz + 1 >= L.nz);
        if (ok) {
            // the row, collapsed over the even axes: C[(dx+1) + 3 (dy+1) + 9 (dz+1)]
            double C[27];
            for (int k = 0; k < 27; ++k) C[k] = 0.0;
            auto put_c = [&](int dx, int dy, int dz, double v) {
                C[(px ? dx + 1 : 1) + 3 * (py ? dy + 1 : 1) + 9 * (pz ? dz + 1 : 1)] += v;
            };
            put_c(0, 0, 0, U[i * M1]);
            for (int j = 0; j < L.m; ++j) {
                const int4 t = L.tab[j];
                if (ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz)
                    put_c(t.x, t.y, t.z, U[i * M1 + j + 1]);
                if (ix - t.x >= 0 && ix - t.x < L.nx && iy - t.y >= 0 && iy - t.y < L.ny && iz - t.z >= 0)
                    put_c(-t.x, -t.y, -t.z, U[(i - t.w) * M1 + j + 1]);
            }
            const double c0 = C[13];
            double acc[8];
            for (int c = 0; c < 8; ++c) acc[c] = 0.0;
            for (int k = 0; k < 27 && ok; ++k) {
                if (k == 13 || C[k] == 0.0) continue;
                const int dx = k % 3 - 1, dy = (k / 3) % 3 - 1, dz = k / 9 - 1;
                const int nxp = ix + dx, nyp = iy + dy, nzp = iz + dz;
                if (nxp < 0 || nxp >= L.nx || nyp < 0 || nyp >= L.ny || nzp < 0 || nzp >= L.nz) continue;
                const int64_t n = nxp + (int64_t)L.nx * (nyp + (int64_t)L.ny * nzp);
                const double f = -C[k] / c0;
                // the neighbour's weights, re-indexed to this node's corners
                for (int cn = 0; cn < 8; ++cn) {
                    const double wn = W[cn * L.N + n];
                    if (wn == 0.0) continue;
                    const int rx = (nxp >> 1) + (cn & 1) - (ix >> 1);
                    const int ry = (nyp >> 1) + ((cn >> 1) & 1) - (iy >> 1);
                    const int rz = (nzp >> 1) + (cn >> 2) - (iz >> 1);
                    if (rx < 0 || rx > 1 || ry < 0 || ry > 1 || rz < 0 || rz > 1) {
                        ok = false;
                        break;
                    }
                    acc[rx + 2 * ry + 4 * rz] += f * wn;
                }
            }
            ok = ok && c0 > 0.0;
            for (int c = 0; c < 8 && ok; ++c) ok = isfinite(acc[c]);
            if (ok)
                for (int c = 0; c < 8; ++c) w[c] = acc[c];
        }
        for (int c = 0; c < 8; ++c) W[c * L.N + i] = w[c];
    }
}

struct SmArgs {
    LvArgs L;
    const double* dinv;  // [nsys][N]
    const double* w;     // [nsys][levels]
    int32_t nlev, lev, nsys;
    const MgScal* sc;    // [nsys][B]
};

// x = w D^{-1} b (the first sweep from zero; on the finest level only at the
// start of a run, elsewhere the kernel that writes b also writes x)
template <int B, typename VT = double>
__global__ __launch_bounds__(kMgT) void k_mg_first(SmArgs a, const double* __restrict__ b, VT* __restrict__ x) {
    const int k = threadIdx.x % B;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        if (!a.sc[sys * B + k].active) continue;
        const double w = a.w[sys * a.nlev + a.lev];
        const int64_t o = sys * a.L.N * B;
        const double* dinv = a.dinv + sys * a.L.N;
        QPAT_MG_ELEMS(e, a.L.N * B) x[o + e] = static_cast<VT>(w * dinv[e / B] * b[o + e]);
    }
}

// y = x + w D^{-1} (b - A x). The systems are swept one after the other by
// the same blocks. DOTS (the last sweep on the finest level, where b = r and
// y = z): also the partial sums r.z, sum z and sum r of every right-hand side,
// of y as stored. x and y in FP64 or FP32 (VT).
template <int KIND, int B, bool DOTS, typename VT = double>
__global__ __launch_bounds__(kMgT) void k_mg_smooth(SmArgs a, const double* __restrict__ b,
                                                    const VT* __restrict__ x, VT* __restrict__ y,
                                                    double* __restrict__ parts) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    __shared__ double sm[(kMgT / 64) * 16];
    const int v = threadIdx.x % Pk<B>::BV;
    const int32_t M1 = a.L.m + 1;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const double w = a.w[sys * a.nlev + a.lev];
        const double* U = rows_of<KIND>(a.L, sys);
        const double* dinv = a.dinv + sys * a.L.N;
        const int64_t o = sys * a.L.N * B + v * V;
        const double* bs = b + o;
        const VT* xs = x + o;
        VT* ys = y + o;
        T rz = 0.0, z1 = 0.0, r1 = 0.0;
        if (pair_active<B>(a.sc, sys, v)) {
            walk<Pk<B>::BV>(a.L.nx, a.L.ny, a.L.nz, [&](int32_t ix, int32_t iy, int32_t iz, int32_t i, int32_t) {
                const T bi = vld<T>(bs + i * B);
                const T ax = apply<KIND, B, VT>(a.L, U, xs, ix, iy, iz, i);
                T yi = vldx<T>(xs + i * B) + (w * dinv[i]) * (bi - ax);
                if constexpr (sizeof(VT) == 4) {
                    static_assert(B == 1, "FP32 sweep output: one right-hand side per thread");
                    yi = held_as<float>(yi);
                }
                vstx<T>(ys + i * B, yi);
                if constexpr (DOTS) {
                    rz += bi * yi;
                    z1 += yi;
                    r1 += bi;
                }
            });
        }
        if constexpr (DOTS) {
            put_sums<B>(parts, sys, 0, rz, sm);
            put_sums<B>(parts, sys, 2, z1, sm);
            put_sums<B>(parts, sys, 3, r1, sm);
        }
    }
}

// r = b - A x (x and r in FP64 or FP32: VT)
template <int KIND, int B, typename VT = double>
__global__ __launch_bounds__(kMgT) void k_mg_resid(SmArgs a, const double* __restrict__ b,
                                                   const VT* __restrict__ x, VT* __restrict__ r) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    const int v = threadIdx.x % Pk<B>::BV;
    const int32_t M1 = a.L.m + 1;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        if (!pair_active<B>(a.sc, sys, v)) continue;
        const double* U = rows_of<KIND>(a.L, sys);
        const int64_t o = sys * a.L.N * B + v * V;
        const double* bs = b + o;
        const VT* xs = x + o;
        VT* rs = r + o;
        walk<Pk<B>::BV>(a.L.nx, a.L.ny, a.L.nz, [&](int32_t ix, int32_t iy, int32_t iz, int32_t i, int32_t) {
            vstx<T>(rs + i * B, vld<T>(bs + i * B) - apply<KIND, B, VT>(a.L, U, xs, ix, iy, iz, i));
        });
    }
}

// the two coarse nodes (or one) whose support holds fine node i along an
// axis: J0 = i / 2 (weight 1 if i is even, 1/2 if odd) and J0 + 1 (1/2 if odd)
struct Span {
    int32_t j0, j1;
    double w0, w1;
    __device__ __forceinline__ Span(int32_t i, int32_t c) {
        j0 = i >> 1;
        const bool odd = i & 1;
        j1 = min(j0 + (odd ? 1 : 0), c - 1);
        w0 = odd ? 0.5 : 1.0;
        w1 = odd ? 0.5 : 0.0;
    }
};

// bc = P^T r on the coarse level c, and the first sweep there, xc = w D^{-1} bc
// (r in FP64 or FP32: RT).
// Fine nodes 2 I + {-1, 0, 1} per axis, weights 1/2, 1, 1/2 (trilinear) or
// from Wc ([nsys][WPack size], operator-dependent, packed); the ones past the
// lattice get weight 0 (their loads are clamped inside it).
template <int B, bool OPW, typename RT = double>
__global__ __launch_bounds__(kMgT) void k_mg_restrict(SmArgs c, int32_t nx, int32_t ny, int32_t nz,
                                                      const RT* __restrict__ r, double* __restrict__ bc,
                                                      double* __restrict__ xc, const float* __restrict__ Wc) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    const int v = threadIdx.x % Pk<B>::BV;
    const int64_t Nf = (int64_t)nx * ny * nz, Nc = c.L.N;
    const WPack pk{nx, ny, nz};
    for (int sys = blockIdx.y; sys < c.nsys; sys += gridDim.y) {
        if (!pair_active<B>(c.sc, sys, v)) continue;
        const double w = c.w[sys * c.nlev + c.lev];
        const double* dinv = c.dinv + sys * Nc;
        const RT* rs = r + sys * Nf * B + v * V;
        const float* Ws = OPW ? Wc + sys * pk.size() : nullptr;
        const int64_t oc = sys * Nc * B + v * V;
        walk<Pk<B>::BV>(c.L.nx, c.L.ny, c.L.nz, [&](int32_t Ix, int32_t Iy, int32_t Iz, int32_t I, int32_t) {
            int32_t fx[3], fy[3], fz[3];
            double wx[3], wy[3], wz[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int32_t gx = 2 * Ix + d - 1, gy = 2 * Iy + d - 1, gz = 2 * Iz + d - 1;
                const double wd = d == 1 ? 1.0 : 0.5;
                wx[d] = gx >= 0 && gx < nx ? wd : 0.0;
                wy[d] = gy >= 0 && gy < ny ? wd : 0.0;
                wz[d] = gz >= 0 && gz < nz ? wd : 0.0;
                fx[d] = min(max(gx, 0), nx - 1);
                fy[d] = min(max(gy, 0), ny - 1);
                fz[d] = min(max(gz, 0), nz - 1);
            }
            // the 27 fine values (and weights) first (clamped indices, all loads
            // in flight together: the tiny levels are latency-bound), then the
            // sum in the order dz, dy, dx
            T fv[27];
            float wv[OPW ? 27 : 1];
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const int32_t row = nx * (fy[dy] + ny * fz[dz]);
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        const int k = (dz * 3 + dy) * 3 + dx;
                        fv[k] = vldx<T>(rs + (row + fx[dx]) * B);
                        // I is corner (d == 0 per axis) of fine node 2 I + d - 1, which is
                        // odd along each such axis: the packed entry exists where the
                        // node is inside the lattice (elsewhere the weight is 0 and the
                        // load, clamped, is not used)
                        if constexpr (OPW)
                            wv[k] = Ws[pk.atc((dx == 0) + 2 * (dy == 0) + 4 * (dz == 0), fx[dx], fy[dy], fz[dz])];
                    }
                }
            __builtin_amdgcn_sched_barrier(0);
            T s = 0.0;
#pragma unroll
            for (int dz = 0; dz < 3; ++dz)
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const double wyz = wy[dy] * wz[dz];
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx) {
                        double wgt = wyz * wx[dx];
                        if constexpr (OPW)
                            if (wgt != 0.0) wgt = static_cast<double>(wv[(dz * 3 + dy) * 3 + dx]);
                        s += wgt * fv[(dz * 3 + dy) * 3 + dx];
                    }
                }
            vst<T>(bc + oc + I * B, s);
            vst<T>(xc + oc + I * B, (w * dinv[I]) * s);
        });
    }
}

// x = base + P xc on fine level f (coarse lattice cx, cy, cz). base = x, or
// with FIRST the first sweep w D^{-1} b, which is then never stored. P:
// trilinear, or the packed weights Wc ([nsys][WPack size]).
template <int B, bool FIRST, bool OPW, bool XF = false>
__global__ __launch_bounds__(kMgT) void k_mg_prolong(SmArgs f, int32_t cx, int32_t cy, int32_t cz,
                                                     const double* __restrict__ xc, const double* __restrict__ b,
                                                     double* __restrict__ x, const float* __restrict__ Wc) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    const int v = threadIdx.x % Pk<B>::BV;
    const int64_t Nf = f.L.N, Nc = (int64_t)cx * cy * cz;
    for (int sys = blockIdx.y; sys < f.nsys; sys += gridDim.y) {
        if (!pair_active<B>(f.sc, sys, v)) continue;
        const double w = f.w[sys * f.nlev + f.lev];
        const double* dinv = f.dinv + sys * Nf;
        const double* xs = xc + sys * Nc * B + v * V;
        const double* bs = b + sys * Nf * B + v * V;
        double* xf = x + sys * Nf * B + v * V;
        float* xf32 = reinterpret_cast<float*>(x) + sys * Nf * B + v * V;   // XF: the fine x in FP32
        const WPack pk{f.L.nx, f.L.ny, f.L.nz};
        const float* Ws = OPW ? Wc + sys * pk.size() : nullptr;
        walk<Pk<B>::BV>(f.L.nx, f.L.ny, f.L.nz, [&](int32_t ix, int32_t iy, int32_t iz, int32_t i, int32_t) {
            const Span sx(ix, cx), sy(iy, cy), sz(iz, cz);
            const int32_t jx[2] = {sx.j0, sx.j1}, jy[2] = {sy.j0, sy.j1}, jz[2] = {sz.j0, sz.j1};
            const double wx[2] = {sx.w0, sx.w1}, wy[2] = {sy.w0, sy.w1}, wz[2] = {sz.w0, sz.w1};
            T s;
            if constexpr (FIRST)
                s = (w * dinv[i]) * vld<T>(bs + i * B);
            else if constexpr (XF)
                s = vldf<T>(xf32 + i * B);
            else
                s = vld<T>(xf + i * B);
            // the 8 coarse values (and weights) first, all loads in flight together
            T cv[8];
            double wgt[8];
#pragma unroll
            for (int c2 = 0; c2 < 2; ++c2)
#pragma unroll
                for (int b2 = 0; b2 < 2; ++b2) {
                    const int32_t row = cx * (jy[b2] + cy * jz[c2]);
                    const double wyz = wy[b2] * wz[c2];
#pragma unroll
                    for (int a2 = 0; a2 < 2; ++a2) {
                        // corner (a2, b2, c2) from J0 = (ix/2, iy/2, iz/2); Span
                        // clamps the index of a zero-weight corner
                        const int cn = a2 + 2 * b2 + 4 * c2;
                        if constexpr (OPW)
                            wgt[cn] = static_cast<double>(Ws[pk.atc(cn, ix, iy, iz)]);
                        else
                            wgt[cn] = wyz * wx[a2];
                        cv[cn] = vld<T>(xs + (row + jx[a2]) * B);
                    }
                }
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (OPW)
#pragma unroll
                for (int cn = 0; cn < 8; ++cn)
                    if (!WPack::held(cn, ix, iy, iz)) wgt[cn] = 0.0;
#pragma unroll
            for (int cn = 0; cn < 8; ++cn) s += wgt[cn] * cv[cn];
            if constexpr (XF)
                vstf<T>(xf32 + i * B, s);
            else
                vst<T>(xf + i * B, s);
        });
    }
}

// x = Ainv b on the coarsest level: one wavefront per output (system, row,
// thread-in-node), its lanes splitting the row and summing by shuffles
template <int B>
__global__ __launch_bounds__(kMgT) void k_mg_dense(int64_t Nc, int nsys, const double* __restrict__ ainv,
                                                   const double* __restrict__ b, double* __restrict__ x,
                                                   const MgScal* __restrict__ sc) {
    // block: kMgT / 64 rows (one per wavefront) of system blockIdx.z for the
    // thread-in-node pair blockIdx.y; that pair's column of b is staged in LDS
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    extern __shared__ __align__(16) unsigned char mg_smem[];
    T* bl = reinterpret_cast<T*>(mg_smem);   // [Nc]
    const int sys = blockIdx.z, v = blockIdx.y;
    if (!pair_active<B>(sc, sys, v)) return;   // uniform over the block
    const double* bs = b + sys * Nc * B + v * V;
#pragma unroll 4
    for (int64_t J = threadIdx.x; J < Nc; J += kMgT) bl[J] = vld<T>(bs + J * B);
    __syncthreads();
    const int lane = threadIdx.x & 63;
    const int64_t I = blockIdx.x * (int64_t)(kMgT / 64) + (threadIdx.x >> 6);
    if (I >= Nc) return;   // whole wavefronts, after the barrier
    const double* A = ainv + (sys * Nc + I) * Nc;
    T s = 0.0;
#pragma unroll 4   // several rows' loads in flight (the coarsest solve is latency-bound)
    for (int64_t J = lane; J < Nc; J += 64) s += A[J] * bl[J];
    double out[V];
#pragma unroll
    for (int c = 0; c < V; ++c) {
        double t = comp(s, c);
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
        out[c] = t;
    }
    if (lane == 0) {
        double* xs = x + sys * Nc * B + v * V + I * B;
#pragma unroll
        for (int c = 0; c < V; ++c) xs[c] = out[c];
    }
}

// ---------------------------------------------------------------- PCG kernels
// The direction ping-pongs between two buffers (po: the last iteration's,
// pn: this one's), so that the fused direction + product kernel can read the
// old direction in the halo of a tile while other blocks write the new one.
struct PcgMg {
    LvArgs L;             // the fine operator
    double* x;            // [nsys][N][B] iterate
    double* r;
    double* po;
    double* pn;
    double* q;
    const double* z;
    double* parts;        // [lanes][4][kMgBlocks]
    MgScal* sc;           // [lanes]
    double rtol2;
    int32_t maxit, deflate, nsys;
    int32_t nb;           // blocks of the kernels that write partials
    // region coarse space (one right-hand side per system), kreg = 0: off;
    // nbr: blocks of the kernels that write the region partials (the later
    // slots hold zeros)
    int32_t kreg, nbr;
    int32_t p32;          // 1: the direction in FP32 on the tiled 16-right-hand-side path (mixed precision)
    int32_t ring;         // kRing: directions and alphas kept in the ring (x formed later), 0: x updated each iteration
    int32_t* slot;        // the ring's iteration counter
    double* ahist;        // [kRing][lanes]
    const int32_t* reg;   // [nsys][N]
    const double* ry;     // [nsys][kRegMax]
    const double* rcorr;  // [nsys][2]: r.(Z y), mean(Z y)
};

// per-component choice between two V-wide values
__device__ __forceinline__ double pick(double a, double b, bool c0, bool) { return c0 ? a : b; }
__device__ __forceinline__ d2v pick(d2v a, d2v b, bool c0, bool c1) {
    d2v r;
    r.x = c0 ? a.x : b.x;
    r.y = c1 ? a.y : b.y;
    return r;
}

// the PCG scalars of thread-in-node v's right-hand sides as V-wide values
template <int B>
struct LaneScal {
    TB<B> alpha, beta, c;
    bool on0, on1;
    __device__ __forceinline__ LaneScal(const MgScal* sc, int sys, int v) {
        const MgScal& s0 = sc[sys * B + v * Pk<B>::V];
        const MgScal& s1 = sc[sys * B + v * Pk<B>::V + Pk<B>::V - 1];
        on0 = s0.active != 0;
        on1 = s1.active != 0;
        if constexpr (Pk<B>::V == 2) {
            alpha = d2v{s0.alpha, s1.alpha};
            beta = d2v{s0.beta, s1.beta};
            c = d2v{s0.c, s1.c};
        } else {
            alpha = s0.alpha;
            beta = s0.beta;
            c = s0.c;
        }
    }
};

// pn = z - c + beta po (right-hand sides that stopped keep pn); ZF: z in FP32
template <int B, bool ZF = false>
__global__ __launch_bounds__(kMgT) void k_mgp_dir(PcgMg a) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V, BV = Pk<B>::BV;
    const int v = threadIdx.x % BV;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const LaneScal<B> s(a.sc, sys, v);
        if (!s.on0 && !s.on1) continue;
        const int64_t o = sys * a.L.N * B + v * V;
        QPAT_MG_ELEMS(e, a.L.N * BV) {
            const int64_t at = o + (e / BV) * B;
            T zc = ZF ? vldf<T>(reinterpret_cast<const float*>(a.z) + at) : vld<T>(a.z + at);
            if constexpr (B == 1) {   // the region coarse-space part of z, y_reg(i) - ybar
                if (a.kreg > 0) {
                    const int32_t rg = a.reg[sys * a.L.N + e];
                    zc += (rg >= 0 ? a.ry[sys * kRegMax + rg] : 0.0) - a.rcorr[2 * sys + 1];
                }
            }
            const T pn = zc - s.c + s.beta * vld<T>(a.po + at);
            vst<T>(a.pn + at, s.on0 && s.on1 ? pn : pick(pn, vld<T>(a.pn + at), s.on0, s.on1));
        }
    }
}

// q = A pn, partial pn.q
template <int KIND, int B>
__global__ __launch_bounds__(kMgT) void k_mgp_spmv(PcgMg a) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    __shared__ double sm[(kMgT / 64) * 16];
    const int v = threadIdx.x % Pk<B>::BV;
    const int32_t M1 = a.L.m + 1;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const double* U = rows_of<KIND>(a.L, sys);
        const int64_t o = sys * a.L.N * B + v * V;
        const double* ps = a.pn + o;
        double* qs = a.q + o;
        T pq = 0.0;
        if (pair_active<B>(a.sc, sys, v)) {
            walk<Pk<B>::BV>(a.L.nx, a.L.ny, a.L.nz, [&](int32_t ix, int32_t iy, int32_t iz, int32_t i, int32_t) {
                const T qi = apply<KIND, B>(a.L, U, ps, ix, iy, iz, i);
                vst<T>(qs + i * B, qi);
                pq += vld<T>(ps + i * B) * qi;
            });
        }
        put_sums<B>(a.parts, sys, 0, pq, sm);
    }
}

// x += alpha pn, r -= alpha q (right-hand sides that stopped keep both),
// partial r.r
template <int B>
__global__ __launch_bounds__(kMgT) void k_mgp_update(PcgMg a) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V, BV = Pk<B>::BV;
    __shared__ double sm[(kMgT / 64) * 16];
    const int v = threadIdx.x % BV;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const LaneScal<B> s(a.sc, sys, v);
        const int64_t o = sys * a.L.N * B + v * V;
        T rr = 0.0;
        if (s.on0 || s.on1) {
            QPAT_MG_ELEMS(e, a.L.N * BV) {
                const int64_t at = o + (e / BV) * B;
                const T p = vld<T>(a.pn + at), r = vld<T>(a.r + at), x = vld<T>(a.x + at);
                const T rn = pick(r - s.alpha * vld<T>(a.q + at), r, s.on0, s.on1);
                vst<T>(a.x + at, pick(x + s.alpha * p, x, s.on0, s.on1));
                vst<T>(a.r + at, rn);
                rr += rn * rn;
            }
        }
        put_sums<B>(a.parts, sys, 1, rr, sm);
    }
}

// deterministic sum of one lane's partials (one block)
__device__ double red(const double* parts, int nb, int lane, int slot, double* sm) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) s += parts[(lane * 4 + slot) * kMgBlocks + b];
    return group_sum<1>(s, sm);
}

// the same sums of three slots of one lane in one pass (each in red's order)
__device__ void red3(const double* parts, int nb, int lane, const int (&slot)[3], double* sm3, double (&out)[3]) {
    double s[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += parts[(lane * 4 + slot[c]) * kMgBlocks + b];
    const int ln = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s[c] += __shfl_xor(s[c], off);
        if (ln == 0) sm3[wave * 3 + c] = s[c];
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double t = 0.0;
        if (threadIdx.x == 0)
            for (int w = 0; w < kMgT / 64; ++w) t += sm3[w * 3 + c];
        out[c] = t;
    }
    __syncthreads();
}

// one block per lane (blockIdx.y). phase 0: alpha = rz / pq; phase 1: rr,
// convergence, iteration count; phase 2 (after the V-cycle): c, beta, rz;
// phase 3: start of a run (after its first V-cycle): c, rz, beta = 0
__global__ __launch_bounds__(kMgT) void k_mgp_scalars(PcgMg a, int phase) {
    __shared__ double sm[kMgT / 64];
    const int lane = blockIdx.y;
    // the direction ring: each iteration's alpha per lane (0 where the lane did
    // not iterate), and the iteration counter, advanced once at the end of an
    // iteration (phase 2, lane 0's block)
    const bool on = a.sc[lane].active != 0;
    if (a.ring > 0 && threadIdx.x == 0) {
        if (phase == 0 && !on) a.ahist[(*a.slot % a.ring) * gridDim.y + lane] = 0.0;
        if (phase == 2 && lane == 0) *a.slot += 1;
    }
    if (!on) return;
    MgScal& s = a.sc[lane];
    if (phase == 0) {
        const double pq = red(a.parts, a.nb, lane, 0, sm);
        if (threadIdx.x == 0) {
            s.pq = pq;
            s.alpha = pq != 0.0 ? s.rz / pq : 0.0;
            if (a.ring > 0) a.ahist[(*a.slot % a.ring) * gridDim.y + lane] = s.alpha;
        }
    } else if (phase == 1) {
        const double rr = red(a.parts, a.nb, lane, 1, sm);
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
        __shared__ double sm3[(kMgT / 64) * 3];
        double v[3];
        red3(a.parts, a.nb, lane, {0, 2, 3}, sm3, v);
        double rz = v[0];
        const double z1 = v[1], r1 = v[2];
        if (threadIdx.x == 0) {
            // z = V(r) + Z y; with deflation its mean is mean(V(r)) + ybar, and the
            // direction takes (V(r) - mean V(r)) + (Z y - ybar): the large, nearly
            // constant part of Z y never passes through the sum with V(r)
            double ybar = 0.0;
            if (a.kreg > 0) {
                rz += a.rcorr[2 * lane];
                ybar = a.rcorr[2 * lane + 1];
            }
            const double c = a.deflate ? z1 / static_cast<double>(a.L.N) : 0.0;
            rz -= (c + ybar) * r1;     // r.(z - mean z)
            s.c = c;
            s.beta = (phase == 2 && s.rz != 0.0) ? rz / s.rz : 0.0;
            s.rz = rz;
        }
    }
}

// ---------------------------------------------------------- region coarse space
// Partial sums of Z^T r (one right-hand side per system): every thread adds
// its nodes into kRegMax register accumulators, then fixed-order block sums.
__global__ __launch_bounds__(kMgT) void k_reg_rsum(PcgMg a, double* __restrict__ rparts) {
    __shared__ double sm[(kMgT / 64) * kRegMax];
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        if (!a.sc[sys].active) continue;   // uniform over the block
        double acc[kRegMax];
#pragma unroll
        for (int j = 0; j < kRegMax; ++j) acc[j] = 0.0;
        const int32_t* rg = a.reg + sys * a.L.N;
        const double* r = a.r + sys * a.L.N;
        // grid-stride order, four nodes' loads in flight per trip
        const int64_t n = a.L.N, stride = (int64_t)gridDim.x * kMgT;
        for (int64_t i0 = blockIdx.x * (int64_t)kMgT + threadIdx.x; i0 < n; i0 += 4 * stride) {
            int32_t g[4];
            double v[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t i = i0 + q * stride;
                g[q] = i < n ? rg[i] : -1;
                v[q] = i < n ? r[i] : 0.0;
            }
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int j = 0; j < kRegMax; ++j) acc[j] += g[q] == j ? v[q] : 0.0;
        }
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
        for (int j = 0; j < kRegMax; ++j) {
            double t = acc[j];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off);
            if (lane == 0) sm[wave * kRegMax + j] = t;
        }
        __syncthreads();
        if (threadIdx.x < kRegMax) {   // the slots no block owns read 0 (fewer blocks than kMgBlocks)
            double t = 0.0;
            for (int w = 0; w < kMgT / 64; ++w) t += sm[w * kRegMax + threadIdx.x];
            double* p = rparts + (sys * kRegMax + threadIdx.x) * kMgBlocks;
            p[blockIdx.x] = t;
            for (int b = blockIdx.x + gridDim.x; b < kMgBlocks; b += gridDim.x) p[b] = 0.0;
        }
        __syncthreads();
    }
}

// One right-hand side per system: the PCG update fused with the two passes
// that read its new r next. x += alpha p, r -= alpha q (a system that
// stopped keeps both) and the partial r.r; the V-cycle's first sweep on the
// finest level, x0 = w D^{-1} r (FP64 or FP32: XT); and, with the region
// coarse space, the partial sums of Z^T r. Four nodes' loads in flight per trip (buffer loads
// with 32-bit offsets: N 8 < 2^31; past the end they read 0 and the stores
// drop); few, full blocks (kMgGrid), so that each block's reduction of its
// kRegMax region sums is spread over many nodes. Slots of blocks past the
// grid read as zero.
template <typename XT>
__global__ __launch_bounds__(kMgT, 4) void k_mgp_update_first(PcgMg a, SmArgs s, XT* __restrict__ x0,
                                                           double* __restrict__ rparts) {
    __shared__ double sm[(kMgT / 64) * kRegMax];
    const int64_t n = a.L.N, stride = (int64_t)gridDim.x * kMgT;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const MgScal& sc = a.sc[sys];
        const bool regions = a.kreg > 0;
        double rr = 0.0, acc[kRegMax];
#pragma unroll
        for (int j = 0; j < kRegMax; ++j) acc[j] = 0.0;
        if (sc.active) {   // uniform over the grid
            const double alpha = sc.alpha, w = s.w[sys * s.nlev];
            const int64_t o = sys * n;
            const uint32_t nb8 = static_cast<uint32_t>(n) * 8u;
            const auto bp = rsrc(a.pn + o, nb8), bq = rsrc(a.q + o, nb8), bd = rsrc(s.dinv + o, nb8);
            const auto bx = rsrc(a.x + o, nb8), br = rsrc(a.r + o, nb8);
            const auto bs = rsrc(x0 + o, static_cast<uint32_t>(n) * static_cast<uint32_t>(sizeof(XT)));
            const auto bg = rsrc(a.reg + (regions ? o : 0), regions ? nb8 / 2 : 0u);
            for (int64_t i0 = blockIdx.x * (int64_t)kMgT + threadIdx.x; i0 < n; i0 += 4 * stride) {
                double pv[4], qv[4], rv[4], xv[4], dv[4];
                int32_t gv[4];
                uint32_t off[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    off[u] = static_cast<uint32_t>(i0 + u * stride) * 8u;   // >= N 8 past the end
                    pv[u] = bload<double>(bp, off[u]);
                    qv[u] = bload<double>(bq, off[u]);
                    rv[u] = bload<double>(br, off[u]);
                    xv[u] = bload<double>(bx, off[u]);
                    dv[u] = bload<double>(bd, off[u]);
                    gv[u] = regions ? bload<int32_t>(bg, off[u] / 2) : -1;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {   // nodes past the end: all zero, stores dropped
                    const double rn = rv[u] - alpha * qv[u];
                    bstore<double>(bx, off[u], xv[u] + alpha * pv[u]);
                    bstore<double>(br, off[u], rn);
                    bstore<XT>(bs, off[u] / (8u / sizeof(XT)), static_cast<XT>(w * dv[u] * rn));
                    rr += rn * rn;
                    if (regions)
#pragma unroll
                        for (int j = 0; j < kRegMax; ++j) acc[j] += gv[u] == j ? rn : 0.0;
                }
            }
        }
        const double t = group_sum<1>(rr, sm);
        if (threadIdx.x == 0) put(a.parts, sys, 1, t);
        if (regions) {   // fixed-order block sums of the region partials (as k_reg_rsum)
            const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
            for (int j = 0; j < kRegMax; ++j) {
                double v = acc[j];
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
                if (lane == 0) sm[wave * kRegMax + j] = v;
            }
            __syncthreads();
            if (threadIdx.x < kRegMax) {
                double v = 0.0;
                for (int wv = 0; wv < kMgT / 64; ++wv) v += sm[wv * kRegMax + threadIdx.x];
                double* pp = rparts + (sys * kRegMax + threadIdx.x) * kMgBlocks;
                pp[blockIdx.x] = v;
                for (int b = blockIdx.x + gridDim.x; b < kMgBlocks; b += gridDim.x) pp[b] = 0.0;
            }
            __syncthreads();
        }
    }
}

// y = E^{-1} Z^T r and the corrections r.(Z y), mean(Z y) (deflation) of the
// dot products and the direction; one block per system (blockIdx.y)
__global__ __launch_bounds__(kMgT) void k_reg_solve(PcgMg a, const double* __restrict__ rparts,
                                                    const double* __restrict__ einv, const double* __restrict__ rsize,
                                                    double* __restrict__ ry, double* __restrict__ rcorr) {
    __shared__ double zr[kRegMax], yy[kRegMax];
    const int sys = blockIdx.y;
    if (!a.sc[sys].active) return;
    const int t = threadIdx.x;
    {   // fixed-order block sums of the partials, every region in one pass
        // (slots of regions past kreg hold zeros)
        __shared__ double wsum[(kMgT / 64) * kRegMax];
        double s[kRegMax];
#pragma unroll
        for (int j = 0; j < kRegMax; ++j) s[j] = 0.0;
        for (int b = t; b < a.nbr; b += kMgT)
#pragma unroll
            for (int j = 0; j < kRegMax; ++j) s[j] += rparts[(sys * kRegMax + j) * kMgBlocks + b];
        const int lane = t & 63, wave = t >> 6;
#pragma unroll
        for (int j = 0; j < kRegMax; ++j) {
            double v = s[j];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
            if (lane == 0) wsum[wave * kRegMax + j] = v;
        }
        __syncthreads();
        if (t < kRegMax) {
            double v = 0.0;
            for (int w = 0; w < kMgT / 64; ++w) v += wsum[w * kRegMax + t];
            zr[t] = t < a.kreg ? v : 0.0;
        }
        __syncthreads();
    }
    if (t < kRegMax) {
        double y = 0.0;
        for (int b = 0; b < a.kreg; ++b) y += einv[(sys * kRegMax + t) * kRegMax + b] * zr[b];
        yy[t] = t < a.kreg ? y : 0.0;
        ry[sys * kRegMax + t] = yy[t];
    }
    __syncthreads();
    if (t == 0) {   // r.(Z y), and with deflation ybar = mean(Z y)
        double c0 = 0.0, c1 = 0.0;
        for (int j = 0; j < a.kreg; ++j) {
            c0 += yy[j] * zr[j];
            c1 += yy[j] * rsize[sys * kRegMax + j];
        }
        rcorr[2 * sys] = c0;
        rcorr[2 * sys + 1] = a.deflate ? c1 / static_cast<double>(a.L.N) : 0.0;
    }
}

// ---- set-up: connected components of the strong couplings (labels converge
// to the smallest node id of each component), region sizes, E = Z^T A Z

// strong coupling of nodes i and j through a_ij
__device__ __forceinline__ bool strong(double aij, double aii, double ajj) {
    return fabs(aij) > kRegTheta * sqrt(fabs(aii * ajj));
}

__global__ __launch_bounds__(kMgT) void k_reg_init(int32_t* __restrict__ lab, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMgT)
        lab[i] = static_cast<int32_t>(i);
}

// hook: every node and the root of its label take the smallest label among
// its strong neighbours
__global__ __launch_bounds__(kMgT) void k_reg_prop(LvArgs L, int32_t* lab, int32_t* __restrict__ flag) {
    const int M1 = L.m + 1;
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        const double aii = L.U[i * M1];
        const int32_t li = __hip_atomic_load(lab + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int32_t mi = li;
        for (int j = 0; j < L.m; ++j) {
            const int4 t = L.tab[j];
            if (ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz) {
                const int64_t k = i + t.w;
                if (strong(L.U[i * M1 + j + 1], aii, L.U[k * M1]))
                    mi = min(mi, __hip_atomic_load(lab + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
            if (ix - t.x >= 0 && ix - t.x < L.nx && iy - t.y >= 0 && iy - t.y < L.ny && iz - t.z >= 0) {
                const int64_t k = i - t.w;
                if (strong(L.U[k * M1 + j + 1], aii, L.U[k * M1]))
                    mi = min(mi, __hip_atomic_load(lab + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
            }
        }
        if (mi < li) {
            atomicMin(lab + li, mi);
            atomicMin(lab + i, mi);
            *flag = 1;
        }
    }
}

// pointer jumping: lab[i] <- lab[lab[i]]
__global__ __launch_bounds__(kMgT) void k_reg_jump(int32_t* lab, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMgT) {
        const int32_t l = __hip_atomic_load(lab + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t ll = __hip_atomic_load(lab + l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ll < l) atomicMin(lab + i, ll);
    }
}

// component sizes; the lanes of a wavefront that share a label add once
// (one component holds most nodes, so per-node atomics would serialise)
__global__ __launch_bounds__(kMgT) void k_reg_count(const int32_t* __restrict__ lab, int32_t* __restrict__ cnt,
                                                    int64_t N) {
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = blockIdx.x * (int64_t)kMgT; i0 < N; i0 += (int64_t)gridDim.x * kMgT) {
        const int64_t i = i0 + threadIdx.x;
        const int32_t l = i < N ? lab[i] : -1;
        unsigned long long todo = __ballot(l >= 0);
        while (todo) {
            const int leader = __ffsll(static_cast<long long>(todo)) - 1;
            const int32_t ll = __shfl(l, leader);
            const unsigned long long same = __ballot(l == ll) & todo;
            if (lane == leader) atomicAdd(cnt + ll, __popcll(same));
            todo &= ~same;
        }
    }
}

// components with at least kRegMin nodes: (root, size) pairs, in any order
__global__ __launch_bounds__(kMgT) void k_reg_roots(const int32_t* __restrict__ lab, const int32_t* __restrict__ cnt,
                                                    int64_t N, int32_t* __restrict__ list, int32_t* __restrict__ n) {
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMgT) {
        if (lab[i] != i || cnt[i] < kRegMin) continue;
        const int32_t at = atomicAdd(n, 1);
        if (at < kRegList) {
            list[2 * at] = static_cast<int32_t>(i);
            list[2 * at + 1] = cnt[i];
        }
    }
}

__global__ __launch_bounds__(kMgT) void k_reg_assign(const int32_t* __restrict__ lab, int64_t N, int k,
                                                     const int32_t* __restrict__ roots, int32_t* __restrict__ reg) {
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < N; i += (int64_t)gridDim.x * kMgT) {
        int32_t r = -1;
        for (int j = 0; j < k; ++j)
            if (lab[i] == roots[j]) r = j;
        reg[i] = r;
    }
}

// largest |a_ij| (bit pattern of a non-negative double)
__global__ __launch_bounds__(kMgT) void k_reg_absmax(const double* __restrict__ U, int64_t n,
                                                     unsigned long long* __restrict__ out) {
    __shared__ double sm[kMgT / 64];
    double m = 0.0;
    for (int64_t e = blockIdx.x * (int64_t)kMgT + threadIdx.x; e < n; e += (int64_t)gridDim.x * kMgT)
        m = fmax(m, fabs(U[e]));
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kMgT / 64; ++w) m = fmax(m, sm[w]);
        atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(m)));
    }
}

// E = Z^T A Z in fixed point (scale: exact, order-independent integer sums):
// the diagonal entry of every node and each stored upper entry a_ij in both
// (reg i, reg j) and (reg j, reg i)
__global__ __launch_bounds__(kMgT) void k_reg_e(LvArgs L, const int32_t* __restrict__ reg, double scale,
                                                unsigned long long* __restrict__ eint) {
    __shared__ unsigned long long se[kRegMax * kRegMax];
    for (int t = threadIdx.x; t < kRegMax * kRegMax; t += kMgT) se[t] = 0ull;
    __syncthreads();
    const int M1 = L.m + 1;
    auto add = [&](int a, int b, double v) {
        const long long q = llrint(v * scale);
        atomicAdd(se + a * kRegMax + b, static_cast<unsigned long long>(q));
    };
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        const int a = reg[i];
        if (a < 0) continue;
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        add(a, a, L.U[i * M1]);
        for (int j = 0; j < L.m; ++j) {
            const int4 t = L.tab[j];
            if (!(ix + t.x >= 0 && ix + t.x < L.nx && iy + t.y >= 0 && iy + t.y < L.ny && iz + t.z < L.nz)) continue;
            const int b = reg[i + t.w];
            if (b < 0) continue;
            const double v = L.U[i * M1 + j + 1];
            add(a, b, v);
            add(b, a, v);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < kRegMax * kRegMax; t += kMgT)
        if (se[t]) atomicAdd(eint + t, se[t]);
}

// partial sums of b and b.b per lane
template <int B>
__global__ __launch_bounds__(kMgT) void k_mgp_bstats(PcgMg a, const double* __restrict__ b) {
    __shared__ double sm[(kMgT / 64) * 16];
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const int64_t o = sys * a.L.N * B;
        double s1 = 0.0, s2 = 0.0;
        QPAT_MG_ELEMS(e, a.L.N * B) {
            s1 += b[o + e];
            s2 += b[o + e] * b[o + e];
        }
        s1 = group_sum<B>(s1, sm);
        s2 = group_sum<B>(s2, sm);
        if (threadIdx.x < B) {
            put(a.parts, sys * B + threadIdx.x, 2, s1);
            put(a.parts, sys * B + threadIdx.x, 3, s2);
        }
    }
}

__global__ __launch_bounds__(kMgT) void k_mgp_init(PcgMg a, double inv_delta) {
    __shared__ double sm[kMgT / 64];
    const int lane = blockIdx.y;
    if (a.ring > 0 && lane == 0 && threadIdx.x == 0) *a.slot = 0;   // a run's first iteration: slot 0
    const double s1 = red(a.parts, a.nb, lane, 2, sm);
    const double s2 = red(a.parts, a.nb, lane, 3, sm);
    if (threadIdx.x == 0) {
        MgScal& s = a.sc[lane];
        const double mean = a.deflate ? s1 / static_cast<double>(a.L.N) : 0.0;
        s.c = mean;                       // subtracted from b by k_mgp_start
        s.mean = mean * inv_delta;
        s.bnorm2 = s2;
        s.rz = s.pq = s.alpha = s.beta = 0.0;
        s.rr = s2;
        s.iters = 0;
        s.done = s2 == 0.0 ? 1 : 0;       // b = 0: x = 0
        s.active = s2 == 0.0 ? 0 : 1;
    }
}

// The start of a run without deflation or initial guess in one pass: r = b,
// x = 0 and the partial sums of b and b.b that k_mgp_init reduces. (The
// first direction of the tiled path ignores the old direction, beta = 0.)
// With the direction ring x is not written here: its first formation starts
// from zero.
template <int B>
__global__ __launch_bounds__(kMgT) void k_mgp_start0(PcgMg a, const double* __restrict__ b) {
    __shared__ double sm[(kMgT / 64) * 16];
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const int64_t o = sys * a.L.N * B;
        double s1 = 0.0, s2 = 0.0;
        QPAT_MG_ELEMS(e, a.L.N * B) {
            const double v = b[o + e];
            a.r[o + e] = v;
            if (a.ring == 0) a.x[o + e] = 0.0;
            s1 += v;
            s2 += v * v;
        }
        s1 = group_sum<B>(s1, sm);
        s2 = group_sum<B>(s2, sm);
        if (threadIdx.x < B) {
            put(a.parts, sys * B + threadIdx.x, 2, s1);
            put(a.parts, sys * B + threadIdx.x, 3, s2);
        }
    }
}

// b -= mean; r = b; po = 0; x = 0 unless a start is given (and b != 0)
template <int B>
__global__ __launch_bounds__(kMgT) void k_mgp_start(PcgMg a, double* __restrict__ b, int has_x0) {
    const int k = threadIdx.x % B;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const MgScal& s = a.sc[sys * B + k];
        const double m = s.c;
        const bool keep = has_x0 && s.active;
        const int64_t o = sys * a.L.N * B;
        QPAT_MG_ELEMS(e, a.L.N * B) {
            b[o + e] -= m;
            a.r[o + e] = b[o + e];
            if (!keep) a.x[o + e] = 0.0;
            a.po[o + e] = 0.0;
        }
    }
}

// true residual r = b - A x (compensated), partial r.r (also the start of a run from x0)
template <int KIND, int B>
__global__ __launch_bounds__(kMgT) void k_mgp_true(PcgMg a, const double* __restrict__ b) {
    using T = TB<B>;
    constexpr int V = Pk<B>::V;
    __shared__ double sm[(kMgT / 64) * 16];
    const int v = threadIdx.x % Pk<B>::BV;
    const int32_t M1 = a.L.m + 1;
    for (int sys = blockIdx.y; sys < a.nsys; sys += gridDim.y) {
        const double* U = a.L.U + sys * a.L.N * M1;   // upper rows: the compensated sum walks the offset table
        const int64_t o = sys * a.L.N * B + v * V;
        const double* bs = b + o;
        const double* xs = a.x + o;
        double* rs = a.r + o;
        T rr = 0.0;
        walk<Pk<B>::BV>(a.L.nx, a.L.ny, a.L.nz, [&](int32_t ix, int32_t iy, int32_t iz, int32_t i, int32_t) {
            const T bi = vld<T>(bs + i * B);
            T ri;
            if (a.L.m == 7) {   // uniform: the loads of a row all in flight
                if constexpr (V == 2) {
                    ri.x = resid_comp7<B>(a.L, U, xs, bi.x, ix, iy, iz, i);
                    ri.y = resid_comp7<B>(a.L, U, xs + 1, bi.y, ix, iy, iz, i);
                } else {
                    ri = resid_comp7<B>(a.L, U, xs, bi, ix, iy, iz, i);
                }
            } else if constexpr (V == 2) {
                ri.x = resid_comp<B>(a.L, U, xs, bi.x, ix, iy, iz, i);
                ri.y = resid_comp<B>(a.L, U, xs + 1, bi.y, ix, iy, iz, i);
            } else {
                ri = resid_comp<B>(a.L, U, xs, bi, ix, iy, iz, i);
            }
            vst<T>(rs + i * B, ri);
            rr += ri * ri;
        });
        put_sums<B>(a.parts, sys, 1, rr, sm);
    }
}

__global__ __launch_bounds__(kMgT) void k_mgp_true_fin(PcgMg a, int reopen) {
    __shared__ double sm[kMgT / 64];
    const int lane = blockIdx.y;
    const double rr = red(a.parts, a.nb, lane, 1, sm);
    if (threadIdx.x == 0) {
        MgScal& s = a.sc[lane];
        s.rr = rr;
        const bool ok = rr <= a.rtol2 * s.bnorm2;
        s.done = ok ? 1 : 0;
        s.active = (!ok && reopen && s.iters < a.maxit) ? 1 : 0;
        s.rz = 0.0;   // a reopened run restarts its Krylov space from the true residual
    }
}


// x += alpha_j p_j over the ring slots of iterations f ... s - 1, in that order
// (the fused multiply-adds the update would have made one iteration at a
// time), for every element of the [N][B] iterate; lanes with alpha_j = 0 did
// not iterate then and keep x (their slot holds no direction of theirs). A
// thread takes the V elements of one 16-byte load of a direction (4 in FP32,
// 2 in FP64; B is a multiple of V), every slot's load in flight before the
// sums; the alphas of all slots are staged in LDS.
template <typename PT>
__global__ __launch_bounds__(kMgT) void k_mgp_ring_flush(int64_t n, int B, double* __restrict__ x,
                                                         const char* __restrict__ ring, int64_t stride,
                                                         const double* __restrict__ ahist, int lanes, int f, int s,
                                                         int x_zero) {
    constexpr int V = 16 / sizeof(PT);
    typedef PT PV __attribute__((ext_vector_type(V)));
    typedef double XV __attribute__((ext_vector_type(2)));
    __shared__ double al[kRing * kMgLanes];
    for (int i = threadIdx.x; i < kRing * lanes; i += kMgT) al[i] = ahist[i];
    __syncthreads();
    const int64_t nq = n / V;
    for (int64_t q = blockIdx.x * (int64_t)kMgT + threadIdx.x; q < nq; q += (int64_t)gridDim.x * kMgT) {
        const int64_t e0 = q * V;
        const int lane0 = static_cast<int>(e0 % B);
        PV pv[kRing];
#pragma unroll
        for (int t = 0; t < kRing; ++t) {
            const int sl = (f + t) % kRing;
            // each direction element is read once here: non-temporal
            pv[t] = f + t < s ? __builtin_nontemporal_load(reinterpret_cast<const PV*>(ring + sl * stride +
                                                                                        e0 * (int64_t)sizeof(PT)))
                              : PV{};
        }
        double xv[V];
#pragma unroll
        for (int c = 0; c < V; c += 2) {   // x_zero: the run started from x = 0, not yet stored
            const XV t2 = x_zero ? XV{0.0, 0.0} : *reinterpret_cast<const XV*>(x + e0 + c);
            xv[c] = t2.x;
            xv[c + 1] = t2.y;
        }
#pragma unroll
        for (int t = 0; t < kRing; ++t) {
            if (f + t >= s) break;   // uniform
            const double* at = al + ((f + t) % kRing) * lanes + lane0;
#pragma unroll
            for (int c = 0; c < V; ++c) {
                const double a = at[c];
                xv[c] = a != 0.0 ? xv[c] + a * static_cast<double>(pv[t][c]) : xv[c];
            }
        }
#pragma unroll
        for (int c = 0; c < V; c += 2) *reinterpret_cast<XV*>(x + e0 + c) = XV{xv[c], xv[c + 1]};
    }
}

// ------------------------------------------------ LDS-tiled finest-level kernels
// On the finest level of a Kuhn lattice with B >= 8 right-hand sides (the
// K solves) the stencil products run 2.5D-tiled: a work item is a tile of
// (kTHX - 2) x (kTHY - 2) lattice columns over a chunk of planes, and the
// block sweeps the chunk plane by plane with the input vector of three planes
// (plus a one-node halo) and the stored operator rows of the same planes in
// LDS. Every input value then comes from global memory kTHX kTHY /
// ((kTHX - 2)(kTHY - 2)) times per product (the halo) instead of once per row
// that uses it, and the gathers are LDS reads with immediate offsets. The
// work items of one XCD are contiguous bands of tiles. Byte offsets are
// 32-bit buffer offsets: loads outside the lattice return 0, stores there are
// dropped.
constexpr int kTT = 512;                 // threads of the tiled kernels
constexpr int kTHX = 12, kTHY = 10;      // halo'd tile
constexpr int kTHN = kTHX * kTHY;
template <int B>
struct MgTile {
    static constexpr int NPF = (kTHN * B + kTT - 1) / kTT;   // input elements per thread and plane
    static constexpr int NU = (kTHN * 8 + kTT - 1) / kTT;     // operator values per thread and plane
    static constexpr size_t LDS = (size_t)3 * (NPF + NU) * kTT * sizeof(double) + 3 * kTHN * sizeof(double);
};
enum TileMode { kTDirSpmv = 0, kTResidFirst = 1, kTSmoothDots = 2, kTTrue = 3, kTResid = 4, kTApply = 5, kTUpdResid = 6 };

struct TileArgs {
    int32_t nx, ny, nz;
    int32_t tiles_x, tiles_y, zc, items;
    int32_t ld, col;      // `in` is [N][ld], columns col ... col + B - 1 (ld = B, col = 0 but in kTApply)
    double scale;         // kTApply: out = scale A in
    const double* U;      // [N][8] the Kuhn stencil form
    const double* in;     // the vector staged in LDS (see the modes), [N][B]
    const double* in2;    // kTDirSpmv: the old direction
    const double* b;      // right-hand side (kTResid*, kTSmoothDots, kTTrue)
    const double* dinv;   // [N] (kTResidFirst, kTSmoothDots)
    const double* w;      // the level's Jacobi weight (kTResidFirst, kTSmoothDots)
    double* out;
    double* out2;         // kTDirSpmv: the new direction
    double* parts;        // partial sums, [lanes][4][kMgBlocks]
    const MgScal* sc;     // [B]
    double* x3;           // kTUpdResid: the iterate (updated in place; null: x is formed from the ring)
    const double* p3;     // kTUpdResid: the direction
    // kTDirSpmv with ring_n > 0: the old and new directions are the ring slots
    // of iterations slot - 1 and slot (ring_stride bytes apart)
    const int32_t* slot;
    const char* ring;
    int64_t ring_stride;
    int32_t ring_n;
};

// kTDirSpmv: the PCG direction and product, p = in - c + beta in2 (in = z,
//   in2 = the old direction) staged, out2 = p, out = A p, partial p.out.
// kTResidFirst: the V-cycle's first sweep and residual, x = w D^{-1} in
//   (in = r) staged, out = b - A x with b = r.
// kTResid: out = b - A in. kTTrue: the same for every right-hand side,
//   partial out.out (out may be null: the partial only).
// kTSmoothDots: out = in + w D^{-1} (b - A in), partial b.out, sum out,
//   sum b (the last finest-level sweep of the V-cycle: b = r, out = z).
// kTApply: out = scale A in for every right-hand side (any Kuhn stencil
//   form U, e.g. the derivative of K in the Jacobian product).
// kTUpdResid: the PCG update fused with kTResidFirst: r' = in - alpha in2
//   (in = r, in2 = q = A p) staged, to out2, x3 += alpha p3, partial r'.r',
//   and out = r' - A x with the first sweep x = w D^{-1} r' (w / a_jj from
//   LDS per neighbour). r' goes to another buffer than r: neighbouring tiles
//   still read r's halo.
// Z32 (kTDirSpmv only): `in` (z, the V-cycle's output) is FP32 [N][B].
// P32 (kTDirSpmv, kTUpdResid): the PCG direction p is stored in FP32. The
// direction kernel rounds p before staging it, so q = A p is the FP64 product of
// exactly the stored p, and the update adds alpha times that same p to the FP64
// iterate: x and r stay consistent (r = b - A x up to FP64 rounding), and the
// rounding only perturbs the choice of the next direction.
template <int MODE, int B, bool Z32 = false, bool P32 = false>
__global__ __launch_bounds__(kTT, 4) void k_mg_tile(TileArgs g) {
    using TL = MgTile<B>;
    constexpr int NPF = TL::NPF, NU = TL::NU, RS = NPF * kTT, US = NU * kTT;
    constexpr int TX = kTHX - 2, TY = kTHY - 2, M1 = 8;
    constexpr uint32_t SZ = sizeof(double);
    constexpr bool UPD = MODE == kTUpdResid;
    // the finest level's residual for the restriction is stored in FP32 (it only
    // feeds the coarse levels of the preconditioner)
    constexpr bool RES32 = MODE == kTResidFirst || MODE == kTResid || UPD;
    constexpr bool HAS_B = MODE != kTDirSpmv && MODE != kTApply && !UPD;
    constexpr bool CENTER_D = MODE == kTSmoothDots;
    // the right-hand side's loads go out a plane ahead where the registers allow
    constexpr bool PRE_B = HAS_B && !CENTER_D;
    extern __shared__ __align__(16) unsigned char mg_smem[];
    __shared__ double sm[(kTT / 64) * 16];
    double* ring = reinterpret_cast<double*>(mg_smem);   // [3][RS]: [halo node][B]
    double* ust = ring + 3 * RS;                          // [3][US]: [halo node][8]
    double* dring = ust + 3 * US;                         // UPD: [3][kTHN] w / a_ii of the halo nodes
    const int tid = threadIdx.x, k = tid % B;
    constexpr bool ALL = MODE == kTTrue || MODE == kTApply;   // every right-hand side, no PCG scalars
    if constexpr (!ALL) {   // every right-hand side stopped: nothing to do
        bool any = false;
        for (int j = 0; j < B; ++j) any = any || g.sc[j].active != 0;
        if (!any) return;
    }
    bool act = true;
    double cc_ = 0.0, beta = 0.0, alpha = 0.0;
    if constexpr (!ALL) {
        const MgScal scl = g.sc[k];
        act = scl.active != 0;
        if constexpr (MODE == kTDirSpmv) {
            cc_ = scl.c;
            beta = scl.beta;
        }
        if constexpr (UPD) alpha = scl.alpha;
    }
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny;
    const uint32_t pv = nxy * B * SZ, pu = nxy * M1 * SZ, pd = nxy * SZ, pin = nxy * g.ld * SZ;
    const double w = (MODE == kTSmoothDots || MODE == kTResidFirst || UPD) ? *g.w : 0.0;
    auto plane = [&](const auto* base, int pl, uint32_t stride, uint32_t bytes) {
        const bool in = pl >= 0 && pl < nz;
        return rsrc(base + (in ? (int64_t)pl * stride : 0), in ? bytes : 0u);
    };
    if constexpr (MODE == kTDirSpmv) {
        if (g.ring_n > 0) {   // this iteration's slot and the one before (uniform)
            const int32_t sl = *g.slot;
            g.in2 = reinterpret_cast<const double*>(g.ring + ((sl + g.ring_n - 1) % g.ring_n) * g.ring_stride);
            g.out2 = reinterpret_cast<double*>(const_cast<char*>(g.ring + (sl % g.ring_n) * g.ring_stride));
        }
    }
    static_assert(!Z32 || MODE == kTDirSpmv, "FP32 input only for the direction + product");
    static_assert(!P32 || MODE == kTDirSpmv || MODE == kTUpdResid, "FP32 direction: direction and update only");
    // LDS node of output slot u (slots past the tile point at an interior node)
    int32_t oc[NPF];
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
        const int nl = (tid + u * kTT) / B;
        oc[u] = nl < TX * TY ? (nl / TX + 1) * kTHX + nl % TX + 1 : kTHX + 1;
    }
    double fr[NPF], f2[NPF], fu[NU], dd = 0.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;

    const int32_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int32_t wx = (g.items + 7) / 8;
    const int32_t it_end = min(g.items, (xcd + 1) * wx);
    const int32_t tiles = g.tiles_x * g.tiles_y;
    for (int32_t item = xcd * wx + slot; item < it_end; item += per) {
        const int32_t ch = item / tiles, t2 = item % tiles;
        const int32_t x0 = (t2 % g.tiles_x) * TX, y0 = (t2 / g.tiles_x) * TY;
        const int32_t zb = ch * g.zc, ze = min(zb + g.zc, nz);
        uint32_t fo[NPF], oo[NPF], od[NPF], uo[NU];
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
            const int nl = (tid + u * kTT) / B;
            const int gx = x0 - 1 + nl % kTHX, gy = y0 - 1 + nl / kTHX;
            const bool fin = nl < kTHN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            fo[u] = fin ? (static_cast<uint32_t>(gy * nx + gx) * g.ld + g.col + k) * SZ : kOut;
            const int ox = x0 + nl % TX, oy = y0 + nl / TX;
            const bool oin = nl < TX * TY && ox < nx && oy < ny;
            oo[u] = oin ? (static_cast<uint32_t>(oy * nx + ox) * B + k) * SZ : kOut;
            od[u] = oin ? static_cast<uint32_t>(oy * nx + ox) * SZ : kOut;
        }
        uint32_t dof = kOut;   // UPD: thread tid < kTHN loads 1 / a_ii of halo node tid
        if (UPD && tid < kTHN) {
            const int gx = x0 - 1 + tid % kTHX, gy = y0 - 1 + tid / kTHX;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) dof = static_cast<uint32_t>(gy * nx + gx) * SZ;
        }
#pragma unroll
        for (int v = 0; v < NU; ++v) {
            const int e = tid + v * kTT, nl = e / M1;
            const int gx = x0 - 1 + nl % kTHX, gy = y0 - 1 + nl / kTHX;
            uo[v] = (nl < kTHN && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
                        ? (static_cast<uint32_t>(gy * nx + gx) * M1 + e % M1) * SZ
                        : kOut;
        }
        auto fetch = [&](int pl) {
            const auto bu = plane(g.U, pl, nxy * M1, pu);
            if constexpr (Z32) {
                const auto bi = plane(reinterpret_cast<const float*>(g.in), pl, nxy * g.ld, pin / 2);
#pragma unroll
                for (int u = 0; u < NPF; ++u)
                    fr[u] = static_cast<double>(bload<float>(bi, fo[u] == kOut ? kOut : fo[u] / 2));
            } else {
                const auto bi = plane(g.in, pl, nxy * g.ld, pin);
#pragma unroll
                for (int u = 0; u < NPF; ++u) fr[u] = bload<double>(bi, fo[u]);
            }
            if constexpr (MODE == kTDirSpmv && P32) {   // the old direction, FP32
                const auto b2 = plane(reinterpret_cast<const float*>(g.in2), pl, nxy * B, pv / 2);
#pragma unroll
                for (int u = 0; u < NPF; ++u)
                    f2[u] = static_cast<double>(bload<float>(b2, fo[u] == kOut ? kOut : fo[u] / 2));
            } else if constexpr (MODE == kTDirSpmv || UPD) {
                const auto b2 = plane(g.in2, pl, nxy * B, pv);
#pragma unroll
                for (int u = 0; u < NPF; ++u) f2[u] = bload<double>(b2, fo[u]);
            }
            if constexpr (MODE == kTResidFirst) {
                const auto bd = plane(g.dinv, pl, nxy, pd);
#pragma unroll
                for (int u = 0; u < NPF; ++u) f2[u] = bload<double>(bd, fo[u] == kOut ? kOut : (fo[u] / SZ - k) / B * SZ);
            }
            if constexpr (UPD) {   // one value per halo node, through LDS (dring)
                const auto bd = plane(g.dinv, pl, nxy, pd);
                dd = bload<double>(bd, dof);
            }
#pragma unroll
            for (int v = 0; v < NU; ++v) fu[v] = bload<double>(bu, uo[v]);
        };
        auto loadb = [&](int z, double(&to)[NPF]) {
            const auto bb = plane(g.b, z, nxy * B, pv);
#pragma unroll
            for (int u = 0; u < NPF; ++u) to[u] = bload<double>(bb, oo[u]);
        };
        double bn[NPF];   // PRE_B: b of the next plane
        if constexpr (PRE_B) loadb(zb, bn);
        auto store = [&](int sl) {
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                double val = fr[u];
                // beta = 0 (a run's first direction) never reads the old direction's values
                if constexpr (MODE == kTDirSpmv)
                    val = fo[u] != kOut ? (beta != 0.0 ? fr[u] - cc_ + beta * f2[u] : fr[u] - cc_) : 0.0;
                if constexpr (MODE == kTDirSpmv && P32) val = static_cast<double>(static_cast<float>(val));
                if constexpr (MODE == kTResidFirst) val = w * f2[u] * fr[u];
                if constexpr (UPD) val = fr[u] - alpha * f2[u];   // r' itself: the sweep scales it per neighbour
                ring[sl * RS + tid + u * kTT] = val;
            }
#pragma unroll
            for (int v = 0; v < NU; ++v) ust[sl * US + tid + v * kTT] = fu[v];
            // w / a_ii of the same plane, with the plane's other staged values:
            // slot sl is free only after the barrier that ends the step before
            if (UPD && tid < kTHN) dring[sl * kTHN + tid] = w * dd;
        };
        // plane z with slots (z, z+1, z-1) = (SZ0, SP0, SL0)
        auto step = [&](int z, auto SZ0, auto SP0, auto SL0) {
            constexpr int sz = decltype(SZ0)::value, sp = decltype(SP0)::value, sl = decltype(SL0)::value;
            store(sp);
            __syncthreads();
            if (z + 1 < ze) fetch(z + 2);
            // per-node inputs of plane z: loads in flight during the arithmetic
            double bc[NPF], dc[NPF];
            if constexpr (PRE_B) {   // loaded one step earlier
#pragma unroll
                for (int u = 0; u < NPF; ++u) bc[u] = bn[u];
                if (z + 1 < ze) loadb(z + 1, bn);
            } else if constexpr (HAS_B) {
                loadb(z, bc);
            }
            if constexpr (CENTER_D) {
                const auto bd = plane(g.dinv, z, nxy, pd);
#pragma unroll
                for (int u = 0; u < NPF; ++u) dc[u] = bload<double>(bd, od[u]);
            }
            constexpr int NO = UPD ? (TX * TY * B + kTT - 1) / kTT : 1;   // output slots in use
            // descriptors stay uniform over the wavefront (a per-lane size would
            // turn every access into a loop over the distinct values); the
            // stores of stopped right-hand sides are skipped by the branch
            // RES32: float [N][B] planes
            // kTTrue with out = null: only the partial out.out (every store dropped)
            const auto bo = RES32 ? rsrc(reinterpret_cast<const float*>(g.out) + (int64_t)z * nxy * B, pv / 2)
                                  : plane(g.out, z, nxy * B, g.out ? pv : 0u);
            if (act) {
                const auto bo2 = (MODE == kTDirSpmv && P32)
                                     ? plane(reinterpret_cast<const float*>(g.out2), z, nxy * B, pv / 2)
                                     : plane(g.out2, z, nxy * B, MODE == kTDirSpmv || UPD ? pv : 0u);
#pragma unroll
                for (int u = 0; u < NPF; ++u) {
                    if (tid + u * kTT >= TX * TY * B) continue;   // whole waves past the tile skip
                    // offsets from the tile-corner neighbour of the node are
                    // non-negative compile-time constants
                    const double* rb = ring + (oc[u] - kTHX - 1) * B + k;
                    const double* ub = ust + (oc[u] - kTHX - 1) * M1;
                    constexpr int cc = kTHX + 1;
                    const double xc = rb[sz * RS + cc * B];
                    double sum = 0.0, rtrue = 0.0;
                    if constexpr (MODE == kTTrue) {   // b - A x, compensated
                        CompSum rc(bc[u]);
                        rc.sub(ub[sz * US + cc * M1], xc);
#pragma unroll
                        for (int j = 0; j < 7; ++j) {
                            const int d = kKy[j] * kTHX + kKx[j];
                            const int up = kKz[j] ? sp : sz, lo = kKz[j] ? sl : sz;
                            rc.sub(ub[sz * US + cc * M1 + j + 1], rb[up * RS + (cc + d) * B]);
                            rc.sub(ub[lo * US + (cc - d) * M1 + j + 1], rb[lo * RS + (cc - d) * B]);
                        }
                        rtrue = rc.value();
                    } else if constexpr (UPD) {   // A (w D^{-1} r'): each neighbour scaled by its w / a_jj
                        const double* db = dring + (oc[u] - kTHX - 1);
                        sum = ub[sz * US + cc * M1] * (db[sz * kTHN + cc] * xc);
#pragma unroll
                        for (int j = 0; j < 7; ++j) {
                            const int d = kKy[j] * kTHX + kKx[j];
                            const int up = kKz[j] ? sp : sz, lo = kKz[j] ? sl : sz;
                            sum += ub[sz * US + cc * M1 + j + 1] * (db[up * kTHN + cc + d] * rb[up * RS + (cc + d) * B]) +
                                   ub[lo * US + (cc - d) * M1 + j + 1] * (db[lo * kTHN + cc - d] * rb[lo * RS + (cc - d) * B]);
                        }
                    } else {
                        sum = ub[sz * US + cc * M1] * xc;
#pragma unroll
                        for (int j = 0; j < 7; ++j) {
                            const int d = kKy[j] * kTHX + kKx[j];
                            const int up = kKz[j] ? sp : sz, lo = kKz[j] ? sl : sz;
                            sum = fma(ub[sz * US + cc * M1 + j + 1], rb[up * RS + (cc + d) * B], sum);
                            sum = fma(ub[lo * US + (cc - d) * M1 + j + 1], rb[lo * RS + (cc - d) * B], sum);
                        }
                    }
                    const bool in = oo[u] != kOut;
                    double o;
                    if constexpr (MODE == kTDirSpmv) {
                        o = sum;
                        a0 += in ? xc * sum : 0.0;
                        if constexpr (P32)   // xc is already an FP32 value
                            bstore_nt_f32(bo2, oo[u] == kOut ? kOut : oo[u] / 2, static_cast<float>(xc));
                        else
                            bstore_nt(bo2, oo[u], xc);   // p: next read by the update pass
                    } else if constexpr (MODE == kTApply) {
                        o = g.scale * sum;
                    } else if constexpr (UPD) {
                        const double rnew = xc;   // the staged r' of the node
                        o = rnew - sum;
                        a1 += in ? rnew * rnew : 0.0;
                        bstore_nt(bo2, oo[u], rnew);
                    } else if constexpr (MODE == kTSmoothDots) {
                        o = xc + w * dc[u] * (bc[u] - sum);
                        a0 += in ? bc[u] * o : 0.0;
                        a1 += in ? o : 0.0;
                        a2 += in ? bc[u] : 0.0;
                    } else {
                        o = MODE == kTTrue ? rtrue : bc[u] - sum;
                        if constexpr (MODE == kTTrue) a1 += in ? o * o : 0.0;
                    }
                    if constexpr (RES32)
                        bstore<float>(bo, oo[u] == kOut ? kOut : oo[u] / 2, static_cast<float>(o));   // read next
                    else
                        bstore_nt(bo, oo[u], o);
                }
                if (UPD && g.x3) {   // x += alpha p on this plane's nodes, after the stencil work
                    __builtin_amdgcn_sched_barrier(0);
                    const auto bx = plane(g.x3, z, nxy * B, pv);
                    if constexpr (P32) {
                        const auto bp = plane(reinterpret_cast<const float*>(g.p3), z, nxy * B, pv / 2);
#pragma unroll
                        for (int u = 0; u < NO; ++u) {
                            if (tid + u * kTT >= TX * TY * B) continue;
                            const double pu = static_cast<double>(bload<float>(bp, oo[u] == kOut ? kOut : oo[u] / 2));
                            bstore_nt(bx, oo[u], bload_nt(bx, oo[u]) + alpha * pu);
                        }
                    } else {
                        const auto bp = plane(g.p3, z, nxy * B, pv);
#pragma unroll
                        for (int u = 0; u < NO; ++u) {
                            if (tid + u * kTT >= TX * TY * B) continue;
                            bstore_nt(bx, oo[u], bload_nt(bx, oo[u]) + alpha * bload_nt(bp, oo[u]));
                        }
                    }
                }
            }
            __syncthreads();
        };
        fetch(zb - 1);
        store(0);
        fetch(zb);
        store(1);
        fetch(zb + 1);
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        for (int z = zb; z < ze; z += 3) {   // plane z - zb + 1 lives in slot (z - zb + 1) % 3
            step(z, I1{}, I2{}, I0{});
            if (z + 1 < ze) step(z + 1, I2{}, I0{}, I1{});
            if (z + 2 < ze) step(z + 2, I0{}, I1{}, I2{});
        }
    }
    auto out_sum = [&](double v, int slot_) {
#pragma unroll
        for (int off = 32; off >= B; off >>= 1) v += __shfl_xor(v, off);
        const int lane = tid & 63, wave = tid >> 6;
        if (lane < B) sm[wave * B + lane] = v;
        __syncthreads();
        if (tid < B) {
            double t = 0.0;
            for (int wv = 0; wv < kTT / 64; ++wv) t += sm[wv * B + tid];
            put(g.parts, tid, slot_, t);
        }
        __syncthreads();
    };
    if constexpr (MODE == kTDirSpmv) out_sum(a0, 0);
    if constexpr (MODE == kTTrue || UPD) out_sum(a1, 1);
    if constexpr (MODE == kTSmoothDots) {
        out_sum(a0, 0);
        out_sum(a1, 2);
        out_sum(a2, 3);
    }
}

// ------------------------------------------------ LDS-tiled restriction
// Finest to first coarse level of the K hierarchy (trilinear weights, B >= 8
// right-hand sides): a work item is a tile of kRX x RY coarse columns over a
// chunk of coarse planes. The block stages each fine plane of the tile's
// support, (2 kRX + 1) x (2 RY + 1) nodes, in LDS with row-contiguous loads
// (double-buffered: the next plane's loads are in flight during the sums)
// and forms the in-plane 3 x 3 weighted sums from LDS; the weights along z
// (1/2 for planes 2K - 1 and 2K + 1, 1 for 2K) are applied as the planes
// stream by, so a fine plane is read once per chunk, the chunk's first plane
// twice. Fine nodes off the lattice load as 0 (their weight is 0).
constexpr int kRX = 8;
template <int B>
struct MgRst {
    static constexpr int RY = kTT / B / kRX;                  // coarse rows per tile (one coarse node per B threads)
    static constexpr int FX = 2 * kRX + 1, FY = 2 * RY + 1;   // fine support of the tile
    static constexpr int NPF = (FX * FY * B + kTT - 1) / kTT;  // fine values per thread and plane
    static constexpr size_t LDS = (size_t)2 * NPF * kTT * sizeof(double);
};

struct RstArgs {
    int32_t nx, ny, nz;      // fine lattice
    int32_t cx, cy, cz;      // coarse lattice
    int32_t tiles_x, tiles_y, zc, items;
    const void* r;           // fine residual [Nf][B], FP64 or (R32) FP32
    const double* dinv;      // coarse 1 / a_ii [Nc]
    const double* w;         // coarse level's Jacobi weight
    double* bc;              // coarse right-hand side [Nc][B]
    double* xc;              // coarse first sweep w D^{-1} bc [Nc][B]
    const MgScal* sc;        // [B]
};

template <int B, bool R32, bool O32 = false>
__global__ __launch_bounds__(kTT) void k_mg_restrict_tile(RstArgs g) {
    using TR = MgRst<B>;
    constexpr int RY = TR::RY, FX = TR::FX, FY = TR::FY, NPF = TR::NPF, RS = NPF * kTT;
    constexpr uint32_t SZ = sizeof(double);
    extern __shared__ __align__(16) unsigned char mg_smem[];
    double* buf = reinterpret_cast<double*>(mg_smem);   // [2][RS]: [support node][B]
    const int tid = threadIdx.x, k = tid % B, cn = tid / B;
    bool any = false;
    for (int j = 0; j < B; ++j) any = any || g.sc[j].active != 0;
    if (!any) return;   // every right-hand side stopped
    const bool act = g.sc[k].active != 0;
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    constexpr uint32_t RZ = R32 ? 4 : 8;   // bytes per fine value
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny, pv = nxy * B * RZ;
    const int64_t cxy = (int64_t)g.cx * g.cy;
    const double wc = *g.w;   // system 0 of the coarse level (the caller passes that entry)
    const int lx = cn % kRX, ly = cn / kRX;
    const int c0 = ((2 * ly + 1) * FX + 2 * lx + 1) * B + k;   // LDS index of the node's centre fine node

    const int32_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int32_t wx = (g.items + 7) / 8;
    const int32_t it_end = min(g.items, (xcd + 1) * wx);
    const int32_t tiles = g.tiles_x * g.tiles_y;
    double fr[NPF];
    for (int32_t item = xcd * wx + slot; item < it_end; item += per) {
        const int32_t ch = item / tiles, t2 = item % tiles;
        const int32_t X0 = (t2 % g.tiles_x) * kRX, Y0 = (t2 / g.tiles_x) * RY;
        const int32_t Kb = ch * g.zc, Ke = min(Kb + g.zc, g.cz);
        uint32_t fo[NPF];
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
            const int e = tid + u * kTT, nl = e / B;
            const int gx = 2 * X0 - 1 + nl % FX, gy = 2 * Y0 - 1 + nl / FX;
            const bool in = nl < FX * FY && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            fo[u] = in ? (static_cast<uint32_t>(gy * nx + gx) * B + e % B) * RZ : kOut;
        }
        auto fetch = [&](int pl) {
            const bool in = pl >= 0 && pl < nz;
            const auto br = rsrc(static_cast<const char*>(g.r) + (in ? (int64_t)pl * pv : 0), in ? pv : 0u);
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                if constexpr (R32)
                    fr[u] = static_cast<double>(bload<float>(br, fo[u]));
                else
                    fr[u] = bload<double>(br, fo[u]);
            }
        };
        auto store = [&](int sl) {
#pragma unroll
            for (int u = 0; u < NPF; ++u) buf[sl * RS + tid + u * kTT] = fr[u];
        };
        auto psum = [&](int sl) {   // in-plane weights 1/2, 1, 1/2 along x and y
            const double* f = buf + sl * RS + c0;
            double rows[3];
#pragma unroll
            for (int dy = -1; dy <= 1; ++dy) {
                const double* q = f + dy * FX * B;
                rows[dy + 1] = 0.5 * (q[-B] + q[B]) + q[0];
            }
            return 0.5 * (rows[0] + rows[2]) + rows[1];
        };
        const int32_t Ix = X0 + lx, Iy = Y0 + ly;
        const bool own = act && Ix < g.cx && Iy < g.cy;
        const int p0 = 2 * Kb - 1, p1 = 2 * Ke - 1;
        fetch(p0);
        store(0);
        double acc = 0.0;
        for (int p = p0; p <= p1; ++p) {
            __syncthreads();
            if (p < p1) fetch(p + 1);
            const double s = psum((p - p0) & 1);
            if (((p - p0) & 1) == 0) {   // odd plane p = 2K - 1 or 2K + 1
                if (p > p0) {            // closes coarse plane K = (p - 1) / 2
                    const double v = acc + 0.5 * s;
                    if (own) {
                        const int64_t I = (int64_t)((p - 1) / 2) * cxy + (int64_t)Iy * g.cx + Ix;
                        if constexpr (O32) {   // the coarse level's vectors in FP32
                            reinterpret_cast<float*>(g.bc)[I * B + k] = static_cast<float>(v);
                            reinterpret_cast<float*>(g.xc)[I * B + k] = static_cast<float>(wc * g.dinv[I] * v);
                        } else {
                            g.bc[I * B + k] = v;
                            g.xc[I * B + k] = wc * g.dinv[I] * v;
                        }
                    }
                }
                acc = 0.5 * s;
            } else {
                acc += s;
            }
            if (p < p1) store((p + 1 - p0) & 1);
        }
        __syncthreads();   // the next item's first store overwrites slot 0
    }
}

// ------------------------------------------------ LDS-tiled 27-point kernels
// The first coarse level of the K hierarchy with 16 right-hand sides: the
// same 2.5D tiling as the finest level (the input vector's planes in LDS),
// with the Galerkin operator's 27-point rows stored whole ([N][kRow27]:
// diagonal, 13 upper, 13 lower entries, zero where the partner is off the
// lattice, padding). The 16 lanes of a node load its row as two 128-byte
// lines, lane k holding entries k and 16 + k, and every entry reaches the
// row's lanes by a DPP row broadcast, so the operator never passes through
// LDS and the partner rows are never gathered.
constexpr int kRow27 = 32;
constexpr int64_t kTile27Min = 16384;   // smaller levels keep the walk kernels (launch-bound anyway)
constexpr int64_t kRow27Min = 131072;   // M_delta: whole 27-point rows pay off from about this size on
enum Tile27Mode { kT27Resid = 0, kT27Smooth = 1 };

// ENTRY: entry-major [27][N] per system (the one-right-hand-side walk
// kernels, row kind 4) instead of node-major [N][kRow27]
template <bool ENTRY>
__global__ __launch_bounds__(kMgT) void k_mg_fullrows27(LvArgs L, double* __restrict__ Uf) {
    const int sys = blockIdx.y;
    constexpr int M1 = 14;
    const double* U = L.U + (int64_t)sys * L.N * M1;
    double* F = Uf + (int64_t)sys * L.N * (ENTRY ? 27 : kRow27);
    for (int64_t i = blockIdx.x * (int64_t)kMgT + threadIdx.x; i < L.N; i += (int64_t)gridDim.x * kMgT) {
        int ix, iy, iz;
        coords(static_cast<int32_t>(i), L.nx, L.ny, ix, iy, iz);
        auto o = [&](int e) -> double& { return ENTRY ? F[e * L.N + i] : F[i * kRow27 + e]; };
        o(0) = U[i * M1];
        for (int j = 0; j < 13; ++j) {
            const int code = 14 + j;
            const int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
            const int64_t lin = dx + (int64_t)L.nx * (dy + (int64_t)L.ny * dz);
            const bool up = ix + dx >= 0 && ix + dx < L.nx && iy + dy >= 0 && iy + dy < L.ny && iz + dz < L.nz;
            const bool lo = ix - dx >= 0 && ix - dx < L.nx && iy - dy >= 0 && iy - dy < L.ny && iz - dz >= 0;
            o(1 + j) = up ? U[i * M1 + 1 + j] : 0.0;
            o(14 + j) = lo ? U[(i - lin) * M1 + 1 + j] : 0.0;
        }
        if constexpr (!ENTRY)
            for (int j = 27; j < kRow27; ++j) o(j) = 0.0;
    }
}

// lane J of each 16-lane row, to the whole row
template <int J>
__device__ __forceinline__ double row_bcast(double v) {
    // one 64-bit DPP move (row_newbcast takes 64-bit operands); every lane is
    // written (row broadcast, full masks), so the old value is never used
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + J, 0xF, 0xF, true);
}

// Two FP32 row entries as one 64-bit value, so that one 64-bit DPP row
// broadcast delivers both: pair = (low: v of this lane, high: v of lane k + 8)
// (row_pair), or two entries stored side by side and loaded as 8 bytes.
__device__ __forceinline__ double row_pair(float v) {
    const int hi = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xF, 0xF, true);   // row_ror:8
    return __builtin_bit_cast(double, (static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                          static_cast<uint32_t>(__builtin_bit_cast(int, v)));
}
__device__ __forceinline__ float pair_lo(double p) {
    return __builtin_bit_cast(float, static_cast<uint32_t>(__builtin_bit_cast(uint64_t, p)));
}
__device__ __forceinline__ float pair_hi(double p) {
    return __builtin_bit_cast(float, static_cast<uint32_t>(__builtin_bit_cast(uint64_t, p) >> 32));
}

// sum over the 13 offset pairs: entry 1 + j (upper) and 14 + j (lower) of
// the row held as (ua: entries 0-15, ub: 16-31) times the LDS neighbours
template <int J>
__device__ __forceinline__ double pair27(double s, double ua, double ub, const double* rb, int sz, int sp,
                                         int sl) {
    constexpr int code = 14 + J;
    constexpr int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
    constexpr int d = (dy * kTHX + dx) * 16;
    const int up = dz ? sp : sz, lo = dz ? sl : sz;
    const double cu = row_bcast<1 + J>(ua);
    double cl;
    if constexpr (14 + J < 16)
        cl = row_bcast<14 + J>(ua);
    else
        cl = row_bcast<J - 2>(ub);
    return fma(cl, rb[lo - d], fma(cu, rb[up + d], s));
}
template <int... J>
__device__ __forceinline__ double apply27(double ua, double ub, const double* rb, int sz, int sp, int sl,
                                          std::integer_sequence<int, J...>) {
    double s = row_bcast<0>(ua) * rb[sz];
    ((s = pair27<J>(s, ua, ub, rb, sz, sp, sl)), ...);
    return s;
}

// the same sum with the row in FP32 pairs: pair k = (entry k, entry k + 16),
// 16 broadcasts for the 27 entries, the products in FP64
template <int... K>
__device__ __forceinline__ void bcast16(double pr, double (&bc)[16], std::integer_sequence<int, K...>) {
    ((bc[K] = row_bcast<K>(pr)), ...);
}
template <int J>
__device__ __forceinline__ double pair27p(double s, const double (&bc)[16], const double* rb, int sz, int sp, int sl) {
    constexpr int code = 14 + J;
    constexpr int dx = code % 3 - 1, dy = (code / 3) % 3 - 1, dz = code / 9 - 1;
    constexpr int d = (dy * kTHX + dx) * 16;
    const int up = dz ? sp : sz, lo = dz ? sl : sz;
    const double cu = static_cast<double>(pair_lo(bc[1 + J]));
    double cl;
    if constexpr (14 + J < 16)
        cl = static_cast<double>(pair_lo(bc[14 + J]));
    else
        cl = static_cast<double>(pair_hi(bc[J - 2]));
    return fma(cl, rb[lo - d], fma(cu, rb[up + d], s));
}
template <int... J>
__device__ __forceinline__ double apply27p(double pr, const double* rb, int sz, int sp, int sl,
                                           std::integer_sequence<int, J...>) {
    double bc[16];
    bcast16(pr, bc, std::make_integer_sequence<int, 16>{});
    double s = static_cast<double>(pair_lo(bc[0])) * rb[sz];
    ((s = pair27p<J>(s, bc, rb, sz, sp, sl)), ...);
    return s;
}

// [n][16][2] FP32 pairs (entry k, entry k + 16) from the [n][kRow27] FP64 rows
__global__ void k_pairs27(int64_t n, const double* __restrict__ U, float* __restrict__ P) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n * 16;
         i += (int64_t)gridDim.x * blockDim.x) {   // (node, k)
        const int64_t node = i / 16, k = i % 16;
        P[2 * i] = static_cast<float>(U[node * kRow27 + k]);
        P[2 * i + 1] = static_cast<float>(U[node * kRow27 + 16 + k]);
    }
}

struct Tile27Args {
    int32_t nx, ny, nz;
    int32_t tiles_x, tiles_y, zc, items;
    const double* Uf;     // [N][kRow27]
    const float* Uf27p;   // R32: the rows as [N][16] FP32 pairs
    const double* x;      // staged vector [N][16]
    const double* b;      // [N][16]
    const double* dinv;   // [N] (kT27Smooth)
    const double* w;      // the level's Jacobi weight (kT27Smooth)
    double* out;          // kT27Resid: b - A x; kT27Smooth: x + w D^{-1} (b - A x)
    const MgScal* sc;     // [16]
};

template <int MODE, bool R32 = false, bool V32 = false>
__global__ __launch_bounds__(kTT, 4) void k_mg_tile27(Tile27Args g) {
    constexpr int B = 16;
    constexpr int NPF = MgTile<B>::NPF, RS = NPF * kTT;
    constexpr int TX = kTHX - 2, TY = kTHY - 2;
    constexpr int NO = (TX * TY * B + kTT - 1) / kTT;   // output slots per thread
    constexpr uint32_t SZ = sizeof(double);
    extern __shared__ __align__(16) unsigned char mg_smem[];
    double* ring = reinterpret_cast<double*>(mg_smem);   // [3][RS]: [halo node][B]
    const int tid = threadIdx.x, k = tid % B;
    bool any = false;
    for (int j = 0; j < B; ++j) any = any || g.sc[j].active != 0;
    if (!any) return;   // every right-hand side stopped
    const bool act = g.sc[k].active != 0;
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny;
    const uint32_t pv = nxy * B * SZ, pr = nxy * kRow27 * SZ, pd = nxy * SZ;
    const double w = MODE == kT27Smooth ? *g.w : 0.0;
    auto plane = [&](const double* base, int pl, uint32_t stride, uint32_t bytes) {
        const bool in = pl >= 0 && pl < nz;
        return rsrc(base + (in ? (int64_t)pl * stride : 0), in ? bytes : 0u);
    };
    // x, b and out of the level: V32 keeps them in FP32 (offsets halve)
    auto vplane = [&](const double* base, int pl) {
        if constexpr (V32) {
            const bool in = pl >= 0 && pl < nz;
            return rsrc(reinterpret_cast<const float*>(base) + (in ? (int64_t)pl * nxy * B : 0), in ? pv / 2 : 0u);
        } else {
            return plane(base, pl, nxy * B, pv);
        }
    };
    auto vload = [&](__amdgpu_buffer_rsrc_t br, uint32_t o) -> double {
        if constexpr (V32)
            return static_cast<double>(bload<float>(br, o == kOut ? kOut : o / 2));
        else
            return bload<double>(br, o);
    };
    int32_t oc[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        const int nl = (tid + u * kTT) / B;
        oc[u] = nl < TX * TY ? (nl / TX + 1) * kTHX + nl % TX + 1 : kTHX + 1;
    }
    double fr[NPF];
    const int32_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int32_t wx = (g.items + 7) / 8;
    const int32_t it_end = min(g.items, (xcd + 1) * wx);
    const int32_t tiles = g.tiles_x * g.tiles_y;
    for (int32_t item = xcd * wx + slot; item < it_end; item += per) {
        const int32_t ch = item / tiles, t2 = item % tiles;
        const int32_t x0 = (t2 % g.tiles_x) * TX, y0 = (t2 / g.tiles_x) * TY;
        const int32_t zb = ch * g.zc, ze = min(zb + g.zc, nz);
        uint32_t fo[NPF], oo[NO], od[NO], ro[NO];
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
            const int nl = (tid + u * kTT) / B;
            const int gx = x0 - 1 + nl % kTHX, gy = y0 - 1 + nl / kTHX;
            const bool fin = nl < kTHN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            fo[u] = fin ? (static_cast<uint32_t>(gy * nx + gx) * B + k) * SZ : kOut;
        }
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int nl = (tid + u * kTT) / B;
            const int ox = x0 + nl % TX, oy = y0 + nl / TX;
            const bool oin = nl < TX * TY && ox < nx && oy < ny;
            oo[u] = oin ? (static_cast<uint32_t>(oy * nx + ox) * B + k) * SZ : kOut;
            od[u] = oin ? static_cast<uint32_t>(oy * nx + ox) * SZ : kOut;
            ro[u] = oin ? (static_cast<uint32_t>(oy * nx + ox) * kRow27 + k) * SZ : kOut;
        }
        auto fetch = [&](int pl) {
            const auto bx = vplane(g.x, pl);
#pragma unroll
            for (int u = 0; u < NPF; ++u) fr[u] = vload(bx, fo[u]);
        };
        auto store = [&](int sl) {
#pragma unroll
            for (int u = 0; u < NPF; ++u) ring[sl * RS + tid + u * kTT] = fr[u];
        };
        // the operator rows and b of plane z, loaded a plane ahead
        double ua[NO], ub[NO], bn[NO];
        auto load_node = [&](int z) {
            const auto bb = vplane(g.b, z);
            if constexpr (R32) {   // the pair (entry k, entry k + 16) as 8 bytes: the layout of a [N][16] vector
                const auto bq = plane(reinterpret_cast<const double*>(g.Uf27p), z, nxy * B, pv);
#pragma unroll
                for (int u = 0; u < NO; ++u) {
                    ua[u] = bload<double>(bq, oo[u]);
                    ub[u] = 0.0;
                    bn[u] = vload(bb, oo[u]);
                }
            } else {
                const auto bu = plane(g.Uf, z, nxy * kRow27, pr);
#pragma unroll
                for (int u = 0; u < NO; ++u) {
                    ua[u] = bload<double>(bu, ro[u]);
                    ub[u] = bload<double>(bu, ro[u] == kOut ? kOut : ro[u] + 16 * SZ);
                    bn[u] = vload(bb, oo[u]);
                }
            }
        };
        load_node(zb);
        auto step = [&](int z, auto SZ0, auto SP0, auto SL0) {
            constexpr int sz = decltype(SZ0)::value, sp = decltype(SP0)::value, sl = decltype(SL0)::value;
            store(sp);
            __syncthreads();
            if (z + 1 < ze) fetch(z + 2);
            double ca[NO], cb[NO], bc[NO], dc[NO];
#pragma unroll
            for (int u = 0; u < NO; ++u) {
                ca[u] = ua[u];
                cb[u] = ub[u];
                bc[u] = bn[u];
            }
            if (z + 1 < ze) load_node(z + 1);
            if constexpr (MODE == kT27Smooth) {   // 1 / a_ii of this plane (one value per node)
                const auto bd = plane(g.dinv, z, nxy, pd);
#pragma unroll
                for (int u = 0; u < NO; ++u) dc[u] = bload<double>(bd, od[u]);
            }
            const auto bo = vplane(g.out, z);   // uniform descriptor; stopped lanes store nowhere
#pragma unroll
            for (int u = 0; u < NO; ++u) {
                if (tid + u * kTT >= TX * TY * B) continue;   // whole waves past the tile skip
                const double* rb = ring + oc[u] * B + k;
                double ax;
                if constexpr (R32)
                    ax = apply27p(ca[u], rb, sz * RS, sp * RS, sl * RS, std::make_integer_sequence<int, 13>{});
                else
                    ax = apply27(ca[u], cb[u], rb, sz * RS, sp * RS, sl * RS, std::make_integer_sequence<int, 13>{});
                double o = bc[u] - ax;
                if constexpr (MODE == kT27Smooth) o = rb[sz * RS] + w * dc[u] * o;
                if constexpr (V32)
                    bstore<float>(bo, act && oo[u] != kOut ? oo[u] / 2 : kOut, static_cast<float>(o));
                else
                    bstore<double>(bo, act ? oo[u] : kOut, o);
            }
            __syncthreads();
        };
        fetch(zb - 1);
        store(0);
        fetch(zb);
        store(1);
        fetch(zb + 1);
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        for (int z = zb; z < ze; z += 3) {   // plane z - zb + 1 lives in slot (z - zb + 1) % 3
            step(z, I1{}, I2{}, I0{});
            if (z + 1 < ze) step(z + 1, I2{}, I0{}, I1{});
            if (z + 2 < ze) step(z + 2, I0{}, I1{}, I2{});
        }
    }
}

// ------------------------------------------------ fused prolongation + last sweep
// The finest level of the K hierarchy with 16 right-hand sides: the staged
// vector of the last sweep is the prolonged correction itself,
// x0 = w D^{-1} r + P x1 (the first sweep recomputed, P trilinear), formed
// plane by plane in LDS from r, 1/a_ii and the coarse planes of the tile's
// support (a 7 x 6 patch of level 1, two coarse planes in LDS), so x0 never
// goes to memory. Then z = x0 + w D^{-1} (r - A x0) with the partial sums
// r.z, sum z, sum r. The stencil rows come whole ([N][16], lane k holds entry
// k) and reach the node's lanes by DPP row broadcasts, which keeps the LDS
// at two blocks per CU. Chunks start on even planes (even zc).
// The sweep is preconditioner work: its rows are read in FP32 and z is stored
// in FP32; the dot products use the stored z, the vector the PCG direction is
// built from. In the FP64 form x0 is staged and A x0 summed in FP64; the FP32
// form (mixed precision) stages x0 in FP32 and sums A x0 in FP32, and forms
// r - A x0 and z in FP64. The PCG vectors themselves and the operator of
// q = A p stay FP64.
constexpr int kPCX = (kTHX - 2) / 2 + 2, kPCY = (kTHY - 2) / 2 + 2;   // coarse patch of a tile
constexpr int kPCN = kPCX * kPCY * 16;                                // its values per coarse plane
struct PSArgs {
    int32_t nx, ny, nz, cx, cy, cz;
    int32_t tiles_x, tiles_y, zc, items;
    const float* Uf;      // [N][16] whole Kuhn rows, FP32
    const double* r;      // [N][16] the PCG residual (level 0's b)
    const double* xc;     // [Nc][16] level 1's solution
    const double* dinv;   // [N]
    const double* w;      // level 0's Jacobi weight
    float* z;             // [N][16], FP32
    double* parts;
    const MgScal* sc;
};

template <int J>
__device__ __forceinline__ double kuhn_pair(double s, double ua, const double* rb, int sz, int sp, int sl) {
    constexpr int d = (kKy[J] * kTHX + kKx[J]) * 16;
    const int up = kKz[J] ? sp : sz, lo = kKz[J] ? sl : sz;
    return fma(row_bcast<8 + J>(ua), rb[lo - d], fma(row_bcast<1 + J>(ua), rb[up + d], s));
}
template <int... J>
__device__ __forceinline__ double apply_kuhn16(double ua, const double* rb, int sz, int sp, int sl,
                                               std::integer_sequence<int, J...>) {
    double s = row_bcast<0>(ua) * rb[sz];
    ((s = kuhn_pair<J>(s, ua, rb, sz, sp, sl)), ...);
    return s;
}

// The FP32 form (mixed precision) of the fused prolongation + sweep stages x0
// in FP32 and sums A x0 in FP32: lane k of a node's 16 holds the row entries k
// and k + 8 as one 64-bit pair (row_pair), so 8 pair broadcasts deliver the
// diagonal, the 7 upper and the 7 lower entries (pair i: entry i low, entry
// i + 8 high).
template <int... J>
__device__ __forceinline__ float apply_kuhn16_f32(double pr, const float* rb, int sz, int sp, int sl,
                                                  std::integer_sequence<int, J...>) {
    static_assert(sizeof...(J) == 7, "the 7 offset pairs of a Kuhn row");
    const double bc[8] = {row_bcast<0>(pr), row_bcast<J + 1>(pr)...};   // pairs 0..7
    float s = pair_lo(bc[0]) * rb[sz];
    // offset J: upper entry 1 + J (pair J + 1, low), lower entry 8 + J (pair J, high)
    auto term = [&](auto JJ) {
        constexpr int j = decltype(JJ)::value;
        constexpr int d = (kKy[j] * kTHX + kKx[j]) * 16;
        const int up = kKz[j] ? sp : sz, lo = kKz[j] ? sl : sz;
        s = fmaf(pair_hi(bc[j]), rb[lo - d], fmaf(pair_lo(bc[j + 1]), rb[up + d], s));
    };
    (term(std::integral_constant<int, J>{}), ...);
    return s;
}

template <bool F32, bool C32 = false>
__global__ __launch_bounds__(kTT, 4) void k_mg_prolong_smooth(PSArgs g) {
    using RT = std::conditional_t<F32, float, double>;   // x0 as staged
    constexpr int B = 16;
    constexpr int NPF = MgTile<B>::NPF, RS = kTHN * B;   // ring slot: exactly the halo tile
    constexpr int TX = kTHX - 2, TY = kTHY - 2;
    constexpr int NO = (TX * TY * B + kTT - 1) / kTT;
    constexpr int NC = (kPCN + kTT - 1) / kTT;   // coarse patch values per thread
    constexpr uint32_t SZ = sizeof(double);
    extern __shared__ __align__(16) unsigned char mg_smem[];
    __shared__ double sm[(kTT / 64) * 16];
    double* dring = reinterpret_cast<double*>(mg_smem);   // [3][kTHN]: 1 / a_ii of the halo nodes
    double* cring = dring + 3 * kTHN;                      // [2][kPCN]: coarse planes, slot Z & 1
    double* rint = cring + 2 * kPCN;                       // [2][TX TY B]: r of the tile's own nodes, slot p & 1
    RT* ring = reinterpret_cast<RT*>(rint + 2 * TX * TY * B);   // [3][RS]: x0 of the halo nodes, [node][16]
    const int tid = threadIdx.x, k = tid % B;
    bool any = false;
    for (int j = 0; j < B; ++j) any = any || g.sc[j].active != 0;
    if (!any) return;
    const bool act = g.sc[k].active != 0;
    const int32_t nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t nxy = static_cast<uint32_t>(nx) * ny, cxy = static_cast<uint32_t>(g.cx) * g.cy;
    const uint32_t pv = nxy * B * SZ, pd = nxy * SZ, pc = cxy * B * SZ;
    const double w = *g.w;
    auto plane = [&](const auto* base, int pl, int n, uint32_t stride, uint32_t bytes) {
        const bool in = pl >= 0 && pl < n;
        return rsrc(base + (in ? (int64_t)pl * stride : 0), in ? bytes : 0u);
    };
    int32_t oc[NO];
#pragma unroll
    for (int u = 0; u < NO; ++u) {
        const int nl = (tid + u * kTT) / B;
        oc[u] = nl < TX * TY ? (nl / TX + 1) * kTHX + nl % TX + 1 : kTHX + 1;
    }
    double fr[NPF], dd = 0.0, cv[NC], cy[NPF];
    bool cy_ok = false;   // cy holds coarse plane (pl + 1) / 2 of the last staged plane pl
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    const int32_t xcd = blockIdx.x & 7, slot = blockIdx.x >> 3, per = gridDim.x >> 3;
    const int32_t wx = (g.items + 7) / 8;
    const int32_t it_end = min(g.items, (xcd + 1) * wx);
    const int32_t tiles = g.tiles_x * g.tiles_y;
    for (int32_t item = xcd * wx + slot; item < it_end; item += per) {
        const int32_t ch = item / tiles, t2 = item % tiles;
        const int32_t x0 = (t2 % g.tiles_x) * TX, y0 = (t2 / g.tiles_x) * TY;
        const int32_t zb = ch * g.zc, ze = min(zb + g.zc, nz);   // zb even
        const int32_t cx0 = x0 / 2 - 1, cy0 = y0 / 2 - 1;        // the patch's first coarse column, row
        uint32_t fo[NPF], o4[NO], dof = kOut;
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
            const int nl = (tid + u * kTT) / B;
            const int gx = x0 - 1 + nl % kTHX, gy = y0 - 1 + nl / kTHX;
            const bool fin = nl < kTHN && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            fo[u] = fin ? (static_cast<uint32_t>(gy * nx + gx) * B + k) * SZ : kOut;
        }
#pragma unroll
        for (int u = 0; u < NO; ++u) {
            const int nl = (tid + u * kTT) / B;
            const int ox = x0 + nl % TX, oy = y0 + nl / TX;
            // the element's byte offset in an FP32 [N][16] array
            o4[u] = nl < TX * TY && ox < nx && oy < ny ? (static_cast<uint32_t>(oy * nx + ox) * B + k) * 4u : kOut;
        }
        if (tid < kTHN) {
            const int gx = x0 - 1 + tid % kTHX, gy = y0 - 1 + tid / kTHX;
            if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) dof = static_cast<uint32_t>(gy * nx + gx) * SZ;
        }
        // the patch's coarse values of this thread (offsets formed at each load)
        auto coarse_off = [&](int u) {
            const int e = tid + u * kTT, cn = e / B;
            const int X = cx0 + cn % kPCX, Y = cy0 + cn / kPCX;
            return e < kPCN && X >= 0 && X < g.cx && Y >= 0 && Y < g.cy
                       ? (static_cast<uint32_t>(Y * g.cx + X) * B + (e % B)) * SZ : kOut;
        };
        // coarse plane Z of level 1's x (C32: stored in FP32)
        auto load_coarse = [&](int Z) {
            if constexpr (C32) {
                const auto bc = plane(reinterpret_cast<const float*>(g.xc), Z, g.cz, cxy * B, pc / 2);
#pragma unroll
                for (int u = 0; u < NC; ++u) {
                    const uint32_t o = coarse_off(u);
                    cv[u] = static_cast<double>(bload<float>(bc, o == kOut ? kOut : o / 2));
                }
            } else {
                const auto bc = plane(g.xc, Z, g.cz, cxy * B, pc);
#pragma unroll
                for (int u = 0; u < NC; ++u) cv[u] = bload<double>(bc, coarse_off(u));
            }
        };
        // fine plane p: r and 1/a_ii; odd p also the coarse plane (p + 1) / 2
        auto fetch = [&](int pl) {
            const auto br = plane(g.r, pl, nz, nxy * B, pv), bd = plane(g.dinv, pl, nz, nxy, pd);
#pragma unroll
            for (int u = 0; u < NPF; ++u) fr[u] = bload<double>(br, fo[u]);
            dd = bload<double>(bd, dof);
            if (pl & 1) load_coarse((pl + 1) / 2);
        };
        auto put_coarse = [&](int Z) {   // coarse plane Z to its slot
#pragma unroll
            for (int u = 0; u < NC; ++u)
                if (tid + u * kTT < kPCN) cring[(Z & 1) * kPCN + tid + u * kTT] = cv[u];
        };
        auto put_d = [&](int sl) {
            if (tid < kTHN) dring[sl * kTHN + tid] = dd;
        };
        // x0 of fine plane pl into ring slot sl (its 1/a_ii already in dring[sl]),
        // with the r of the tile's own nodes (the sweep's b) into rint
        auto store = [&](int sl, int pl) {
            const bool pin = pl >= 0 && pl < nz;
            const int z0 = pl >> 1, z1 = (pl + 1) >> 1;
            const double wz1 = (pl & 1) ? 0.5 : 0.0, wz0 = 1.0 - wz1;
            const double* c0 = cring + (z0 & 1) * kPCN + k;
            const double* c1 = cring + (z1 & 1) * kPCN + k;
            // the bilinear value of coarse plane (pl + 1) / 2 at each element is
            // kept in cy: an odd plane's upper coarse plane is the next even
            // plane's own, so each coarse plane is interpolated once per item
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                const int e = tid + u * kTT, nl = e / B;
                if (e >= RS) continue;
                const int lx = nl % kTHX - 1, ly = nl / kTHX - 1;
                if (lx >= 0 && lx < TX && ly >= 0 && ly < TY) rint[(pl & 1) * (TX * TY * B) + (ly * TX + lx) * B + k] = fr[u];
                double v = 0.0;
                if (pin && fo[u] != kOut) {   // inside the halo tile and the grid
                    v = w * dring[sl * kTHN + nl] * fr[u];
                    const int gx = x0 - 1 + nl % kTHX, gy = y0 - 1 + nl / kTHX;
                    const int o = (((gy >> 1) - cy0) * kPCX + (gx >> 1) - cx0) * B;
                    const int dx = (gx & 1) ? B : 0, dy = (gy & 1) ? kPCX * B : 0;
                    // trilinear weights are 1 or 1/2 per axis: with the even-parity
                    // neighbour read twice, every case is a quarter of a four-term
                    // sum (scaling by powers of two is exact)
                    auto bil = [&](const double* cp) {
                        const double* q = cp + o;
                        return 0.25 * ((q[0] + q[dx]) + (q[dy] + q[dy + dx]));
                    };
                    double b0;
                    if (cy_ok) b0 = cy[u];
                    else b0 = bil(c0);
                    if (pl & 1) {   // odd planes lie halfway between two coarse planes
                        const double b1 = bil(c1);
                        v = fma(wz1, b1, fma(wz0, b0, v));
                        cy[u] = b1;
                    } else {        // even planes on one (weight 1: fma(1, a, b) = a + b exactly)
                        v += b0;
                        cy[u] = b0;
                    }
                }
                ring[sl * RS + e] = static_cast<RT>(v);
                __builtin_amdgcn_sched_barrier(0);   // one element's coarse reads live at a time
            }
            cy_ok = pin;
        };
        auto step = [&](int z, auto SZ0, auto SP0, auto SL0) {
            constexpr int sz = decltype(SZ0)::value, sp = decltype(SP0)::value, sl = decltype(SL0)::value;
            float ua32[NO];   // the rows of this plane's nodes: in flight during the staging
            const auto bu = plane(g.Uf, z, nz, nxy * B, pv / 2);
#pragma unroll
            for (int u = 0; u < NO; ++u) ua32[u] = bload<float>(bu, o4[u]);
            store(sp, z + 1);
            __syncthreads();
            if (z + 1 < ze) fetch(z + 2);
            const auto bo = plane(g.z, z, nz, nxy * B, pv / 2);
#pragma unroll
            for (int u = 0; u < NO; ++u) {
                if (tid + u * kTT >= TX * TY * B) continue;   // whole waves past the tile skip
                const RT* rb = ring + oc[u] * B + k;
                double ax;
                if constexpr (F32)
                    ax = apply_kuhn16_f32(row_pair(ua32[u]), rb, sz * RS, sp * RS, sl * RS,
                                          std::make_integer_sequence<int, 7>{});
                else
                    ax = apply_kuhn16(static_cast<double>(ua32[u]), rb, sz * RS, sp * RS, sl * RS,
                                      std::make_integer_sequence<int, 7>{});
                const double xc = rb[sz * RS];
                const double bcu = rint[(z & 1) * (TX * TY * B) + tid + u * kTT];
                const float o32 = static_cast<float>(xc + w * dring[sz * kTHN + oc[u]] * (bcu - ax));
                const double o = static_cast<double>(o32);
                const bool in = act && o4[u] != kOut;
                a0 += in ? bcu * o : 0.0;
                a1 += in ? o : 0.0;
                a2 += in ? bcu : 0.0;
                bstore_nt_f32(bo, act ? o4[u] : kOut, o32);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (z + 1 < ze) {   // plane z + 2's 1/a_ii (slot sl) and, odd, coarse plane (z + 3) / 2
                put_d(sl);
                if ((z + 2) & 1) put_coarse((z + 3) / 2);
            }
            __syncthreads();
        };
        cy_ok = false;
        load_coarse(zb / 2 - 1);   // staging plane zb - 1 needs coarse planes zb/2 - 1 and zb/2
        put_coarse(zb / 2 - 1);
        fetch(zb - 1);             // odd: also coarse plane zb / 2
        put_d(0);
        put_coarse(zb / 2);
        __syncthreads();
        store(0, zb - 1);
        fetch(zb);
        put_d(1);
        __syncthreads();
        store(1, zb);
        fetch(zb + 1);             // odd: coarse plane zb / 2 + 1
        put_d(2);
        put_coarse(zb / 2 + 1);    // slot of zb/2 - 1, whose last use (plane zb - 1) is staged
        __syncthreads();
        using I0 = std::integral_constant<int, 0>;
        using I1 = std::integral_constant<int, 1>;
        using I2 = std::integral_constant<int, 2>;
        for (int z = zb; z < ze; z += 3) {   // plane z - zb + 1 lives in slot (z - zb + 1) % 3
            step(z, I1{}, I2{}, I0{});
            if (z + 1 < ze) step(z + 1, I2{}, I0{}, I1{});
            if (z + 2 < ze) step(z + 2, I0{}, I1{}, I2{});
        }
    }
    auto out_sum = [&](double v, int slot_) {
#pragma unroll
        for (int off = 32; off >= B; off >>= 1) v += __shfl_xor(v, off);
        const int lane = tid & 63, wave = tid >> 6;
        if (lane < B) sm[wave * B + lane] = v;
        __syncthreads();
        if (tid < B) {
            double t = 0.0;
            for (int wv = 0; wv < kTT / 64; ++wv) t += sm[wv * B + tid];
            put(g.parts, tid, slot_, t);
        }
        __syncthreads();
    };
    out_sum(a0, 0);
    out_sum(a1, 2);
    out_sum(a2, 3);
}
template <bool F32>
constexpr size_t kPSLds = (size_t)(3 * kTHN + 2 * kPCN + 2 * (kTHX - 2) * (kTHY - 2) * 16) * sizeof(double) +
                          (size_t)3 * kTHN * 16 * (F32 ? sizeof(float) : sizeof(double));

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
    a.Uf = L.Uf;
    a.Uf32 = L.Uf32;
    return a;
}

// a multiple of 8 blocks (the XCD row split), at most cap (<= kMgBlocks)
inline dim3 vgrid(int64_t n, int cap = kMgGrid) { return dim3((grid_for(n, kMgT, cap) + 7) & ~7); }

#define QPAT_MG_KIND(kind, B, KERNEL, ...)                                 \
    switch (kind) {                                                         \
        case 1: hipLaunchKernelGGL((KERNEL<1, B>), __VA_ARGS__); break;     \
        case 2: hipLaunchKernelGGL((KERNEL<2, B>), __VA_ARGS__); break;     \
        case 3: hipLaunchKernelGGL((KERNEL<3, B>), __VA_ARGS__); break;     \
        case 4:                                                             \
            if constexpr (B == 1) hipLaunchKernelGGL((KERNEL<4, 1>), __VA_ARGS__); \
            break;                                                          \
        case 5:                                                             \
            if constexpr (B == 1) hipLaunchKernelGGL((KERNEL<5, 1>), __VA_ARGS__); \
            break;                                                          \
        case 6:                                                             \
            if constexpr (B == 1) hipLaunchKernelGGL((KERNEL<6, 1>), __VA_ARGS__); \
            break;                                                          \
        default: hipLaunchKernelGGL((KERNEL<0, B>), __VA_ARGS__); break;    \
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
    // the columns carry independent rounding: make the inverse exactly
    // symmetric, as the preconditioner it is part of must be
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
            A[(size_t)i * n + j] = A[(size_t)j * n + i] = v;
        }
    return true;
}

template <int B, bool DOTS>
void launch_smooth(int kind, dim3 g, hipStream_t st, const SmArgs& a, const double* b, const double* x, double* y,
                   double* parts) {
    switch (kind) {
        case 1: hipLaunchKernelGGL((k_mg_smooth<1, B, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts); break;
        case 2: hipLaunchKernelGGL((k_mg_smooth<2, B, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts); break;
        case 3: hipLaunchKernelGGL((k_mg_smooth<3, B, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts); break;
        case 4:
            if constexpr (B == 1) hipLaunchKernelGGL((k_mg_smooth<4, 1, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts);
            break;
        case 5:
            if constexpr (B == 1) hipLaunchKernelGGL((k_mg_smooth<5, 1, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts);
            break;
        case 6:
            if constexpr (B == 1) hipLaunchKernelGGL((k_mg_smooth<6, 1, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts);
            break;
        default: hipLaunchKernelGGL((k_mg_smooth<0, B, DOTS>), g, dim3(kMgT), 0, st, a, b, x, y, parts); break;
    }
}

// one grid row per system (blockIdx.y) for one right-hand side per thread: the
// systems' sweeps then run side by side instead of one after the other in
// each block (the one-right-hand-side kernels are latency-bound)
inline dim3 sys_rows(dim3 g, int B, int nsys) { return dim3(g.x, B == 1 ? nsys : 1); }

// grid of the stencil and V-cycle kernels of a level with n nodes
template <int B>
dim3 sgrid(int64_t n, int nsys = 1) {
    // one right-hand side per thread (the M_delta solves) is latency-bound: more blocks
    return sys_rows(vgrid(n * Pk<B>::BV, B == 1 ? kMgBlocks : kMgGrid), B, nsys);
}

// the direction ring of the tiled iterations, as the direction kernel reads it
struct RingArg {
    const int32_t* slot = nullptr;
    const char* base = nullptr;
    int64_t stride = 0;
    int32_t n = 0;
};

template <int MODE, int B, bool Z32 = false, bool P32 = false>
void launch_tile(const MgState& M, const TileGeo& t, hipStream_t st, const double* in, const double* in2,
                 const double* b, double* out, double* out2, double* x3 = nullptr, const double* p3 = nullptr,
                 RingArg ring = {}) {
    if constexpr (B >= 8) {   // tile_setup turns the tiling on only there
        const MgLevel& L = M.lv[0];
        TileArgs g;
        g.nx = L.nx;
        g.ny = L.ny;
        g.nz = L.nz;
        g.tiles_x = t.tiles_x;
        g.tiles_y = t.tiles_y;
        g.zc = t.zc;
        g.items = t.items;
        g.ld = B;
        g.col = 0;
        g.scale = 1.0;
        g.U = L.U;
        g.in = in;
        g.in2 = in2;
        g.b = b;
        g.dinv = L.dinv;
        g.w = M.w;   // system 0, level 0
        g.out = out;
        g.out2 = out2;
        g.parts = M.parts;
        g.sc = M.sc;
        g.x3 = x3;
        g.p3 = p3;
        g.slot = ring.slot;
        g.ring = ring.base;
        g.ring_stride = ring.stride;
        g.ring_n = ring.n;
        hipLaunchKernelGGL((k_mg_tile<MODE, B, Z32, P32>), dim3(t.blocks), dim3(kTT), MgTile<B>::LDS, st, g);
    }
}

// coarse level l: out = b - A x (kT27Resid) or x + w D^{-1} (b - A x) (kT27Smooth)
template <int MODE>
void launch_tile27(const MgState& M, const TileGeo& t, int l, hipStream_t st, const double* x, const double* b,
                   double* out, bool v32 = false) {
    const MgLevel& L = M.lv[l];
    const TileGeo::Lv27& q = t.t27[l];
    Tile27Args g;
    g.nx = L.nx;
    g.ny = L.ny;
    g.nz = L.nz;
    g.tiles_x = q.tx;
    g.tiles_y = q.ty;
    g.zc = q.zc;
    g.items = q.items;
    g.Uf = L.Uf;
    g.Uf27p = L.Uf27p;
    g.x = x;
    g.b = b;
    g.dinv = L.dinv;
    g.w = M.w + l;   // system 0, level l
    g.out = out;
    g.sc = M.sc;
    const size_t lds = (size_t)3 * MgTile<16>::NPF * kTT * sizeof(double);
    if (L.Uf27p && v32)   // the rows and (v32) the level's vectors in FP32
        hipLaunchKernelGGL((k_mg_tile27<MODE, true, true>), dim3(q.blocks), dim3(kTT), lds, st, g);
    else if (L.Uf27p)   // the rows in FP32 (the V-cycle's coarse operators)
        hipLaunchKernelGGL((k_mg_tile27<MODE, true>), dim3(q.blocks), dim3(kTT), lds, st, g);
    else
        hipLaunchKernelGGL((k_mg_tile27<MODE, false>), dim3(q.blocks), dim3(kTT), lds, st, g);
}
inline bool tiled27(const TileGeo& t, int l) { return l >= 1 && l < kMgMaxLevels && t.t27[l].on; }

// level 0: z = x0 + w D^{-1} (r - A x0), x0 = w D^{-1} r + P x1 (fused, 16 right-hand sides)
inline void launch_ps(const MgState& M, const TileGeo& t, hipStream_t st, const double* r, const double* x1, double* z,
                      bool f32, bool c32 = false) {
    const MgLevel& L = M.lv[0];
    const MgLevel& C = M.lv[1];
    PSArgs g;
    g.nx = L.nx;
    g.ny = L.ny;
    g.nz = L.nz;
    g.cx = C.nx;
    g.cy = C.ny;
    g.cz = C.nz;
    g.tiles_x = t.tiles_x;
    g.tiles_y = t.tiles_y;
    g.zc = f32 ? t.ps_zc32 : t.ps_zc;
    g.items = f32 ? t.ps_items32 : t.ps_items;
    g.Uf = L.Ufk32;
    g.r = r;
    g.xc = x1;
    g.dinv = L.dinv;
    g.w = M.w;   // system 0, level 0
    g.z = reinterpret_cast<float*>(z);   // FP32 in the double buffer's first half
    g.parts = M.parts;
    g.sc = M.sc;
    if (f32 && c32)   // c32: level 1's x in FP32
        hipLaunchKernelGGL((k_mg_prolong_smooth<true, true>), dim3(t.ps_blocks32), dim3(kTT), kPSLds<true>, st, g);
    else if (f32)
        hipLaunchKernelGGL(k_mg_prolong_smooth<true>, dim3(t.ps_blocks32), dim3(kTT), kPSLds<true>, st, g);
    else if (c32)
        hipLaunchKernelGGL((k_mg_prolong_smooth<false, true>), dim3(t.ps_blocks), dim3(kTT), kPSLds<false>, st, g);
    else
        hipLaunchKernelGGL(k_mg_prolong_smooth<false>, dim3(t.ps_blocks), dim3(kTT), kPSLds<false>, st, g);
}

// level l's residual to level l + 1's b and first sweep xc (tiled; trilinear)
template <int B>
void launch_restrict(const MgState& M, const TileGeo& t, int l, hipStream_t st, double* xc, bool v1 = false) {
    if constexpr (B >= 8) {
        const MgLevel& L = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        const TileGeo::Rst& q = t.rst[l];
        RstArgs g;
        g.nx = L.nx;
        g.ny = L.ny;
        g.nz = L.nz;
        g.cx = C.nx;
        g.cy = C.ny;
        g.cz = C.nz;
        g.tiles_x = q.tx;
        g.tiles_y = q.ty;
        g.zc = q.zc;
        g.items = q.items;
        g.r = L.r;
        g.dinv = C.dinv;
        g.w = M.w + l + 1;   // system 0, level l + 1
        g.bc = C.b;
        g.xc = xc;
        g.sc = M.sc;
        // the finest level's residual comes from the tiled kernels in FP32; v1:
        // level 1's vectors are FP32 too (written here from level 0, read here
        // towards level 2)
        if (l == 0 && v1)
            hipLaunchKernelGGL((k_mg_restrict_tile<B, true, true>), dim3(q.blocks), dim3(kTT), MgRst<B>::LDS, st, g);
        else if (l == 0 || (l == 1 && v1))
            hipLaunchKernelGGL((k_mg_restrict_tile<B, true>), dim3(q.blocks), dim3(kTT), MgRst<B>::LDS, st, g);
        else
            hipLaunchKernelGGL((k_mg_restrict_tile<B, false>), dim3(q.blocks), dim3(kTT), MgRst<B>::LDS, st, g);
    }
}

// The finest-level tiling for block size B: on for the Kuhn stencil of one
// system with B >= 8 whose plane offsets fit 32 bits; the z-chunk length
// balances the work items over the blocks resident per XCD.
// ---- autotuning of the tiled z-chunk length
// The cost model ranks z-chunk lengths by (item waves per XCD) x (planes + 2).
// With opts.autotune the lowest-cost candidates (at most kTuneCands distinct
// lengths) are timed on the device, each by one untimed and kTuneReps timed
// launches of the kernel on scratch vectors, in kTuneRounds interleaved rounds
// (each candidate keeps its fastest round: the first launches of a process run
// on a GPU that is still raising its clocks). The model's first candidate is
// kept unless another is faster by more than kTuneMargin, so timing noise of a
// few percent cannot move the choice away from the model's. The choice is
// cached per process by (kernel, lattice size, block), so a second context on
// the same lattice reuses it; timings taken while other streams load the GPU
// (concurrent batched instances) are noisier but only pick among the model's
// own candidates.
constexpr int kTuneCands = 4, kTuneReps = 3, kTuneRounds = 2;
constexpr float kTuneMargin = 0.02f;

// index of the candidate to keep from their times (model order)
inline size_t tune_pick(const std::vector<float>& ms) {
    size_t best = 0;
    for (size_t i = 1; i < ms.size(); ++i)
        if (ms[i] < ms[0] * (1.f - kTuneMargin) && ms[i] < ms[best]) best = i;
    return best;
}
using TuneKey = std::tuple<int, int, int, int, int>;   // kernel, nx, ny, nz, B
std::mutex g_tune_mu;
std::map<TuneKey, int32_t> g_tune;

// the candidate chunk lengths (even: only even lengths), lowest model cost first
inline std::vector<int64_t> chunk_candidates(int64_t nz, int64_t tiles, int64_t conc, bool even) {
    std::vector<std::pair<int64_t, int64_t>> cz;   // (cost, zc)
    for (int64_t nch = 1; nch <= nz; ++nch) {
        int64_t zc = (nz + nch - 1) / nch;
        if (even) zc += zc & 1;
        const int64_t items = tiles * ((nz + zc - 1) / zc);
        const int64_t cost = (((items + 7) / 8 + conc - 1) / conc) * (zc + 2);
        bool seen = false;
        for (auto& e : cz) seen = seen || e.second == zc;
        if (!seen) cz.emplace_back(cost, zc);
    }
    std::stable_sort(cz.begin(), cz.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
    std::vector<int64_t> out;
    for (size_t i = 0; i < cz.size() && (int)i < kTuneCands; ++i) out.push_back(cz[i].second);
    return out;
}

// mean time (ms) of kTuneReps launches after one untimed launch
template <typename F>
qpat_status time_launches(qpat_ctx* c, F&& launch, float* ms) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QPAT_HIP(c, hipEventCreate(&e0));
    QPAT_HIP(c, hipEventCreate(&e1));
    launch();
    QPAT_HIP(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < kTuneReps; ++r) launch();
    QPAT_HIP(c, hipEventRecord(e1, c->stream));
    QPAT_HIP(c, hipGetLastError());
    QPAT_HIP(c, hipEventSynchronize(e1));
    QPAT_HIP(c, hipEventElapsedTime(ms, e0, e1));
    *ms /= kTuneReps;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return QPAT_OK;
}

template <int B>
qpat_status tile_setup(qpat_ctx* c, MgState& M) {
    TileGeo& t = M.tiles[B];
    if (t.ready) return QPAT_OK;
    t.ready = true;
    t.on = false;
    const MgLevel& L = M.lv[0];
    if constexpr (B >= 8) {
        if (M.nsys != 1 || L.kind != 1 || L.N * B * (int64_t)sizeof(double) >= (int64_t(1) << 31)) return QPAT_OK;
        static_assert(MgTile<B>::LDS <= 159 * 1024, "tiled multigrid LDS budget");
        const void* fns[10] = {reinterpret_cast<const void*>(&k_mg_tile<kTDirSpmv, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTResidFirst, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTSmoothDots, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTTrue, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTResid, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTApply, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTUpdResid, B>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTDirSpmv, B, true>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTDirSpmv, B, true, true>),
                              reinterpret_cast<const void*>(&k_mg_tile<kTUpdResid, B, false, true>)};
        for (const void* f : fns)   // dynamic LDS beyond the default limit is allowed per kernel
            QPAT_HIP(c, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MgTile<B>::LDS));
        int occ = 1, cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, fns[2], kTT, MgTile<B>::LDS) != hipSuccess) occ = 1;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) cus = 256;
        const int64_t blocks = sgrid<B>(L.N).x;
        const int64_t conc = std::max<int64_t>(1, std::min<int64_t>((int64_t)std::max(occ, 1) * (cus / 8), blocks / 8));
        const int64_t tx = (L.nx + kTHX - 3) / (kTHX - 2), ty = (L.ny + kTHY - 3) / (kTHY - 2);
        int64_t best = -1, best_zc = L.nz;
        for (int64_t nch = 1; nch <= L.nz; ++nch) {
            const int64_t zc = (L.nz + nch - 1) / nch;
            const int64_t items = tx * ty * ((L.nz + zc - 1) / zc);
            const int64_t cost = (((items + 7) / 8 + conc - 1) / conc) * (zc + 2);
            if (best < 0 || cost < best) {
                best = cost;
                best_zc = zc;
            }
        }
        t.tiles_x = static_cast<int32_t>(tx);
        t.tiles_y = static_cast<int32_t>(ty);
        auto set_zc = [&](int64_t zc) {
            t.zc = static_cast<int32_t>(zc);
            t.items = static_cast<int32_t>(tx * ty * ((L.nz + zc - 1) / zc));
            t.blocks = static_cast<int32_t>(8 * std::min<int64_t>(conc, (t.items + 7) / 8));
        };
        set_zc(best_zc);
        t.zc_model = t.zc;
        t.on = true;
        if (c->opts.autotune) {
            // time the two kernels of every PCG iteration that share this geometry, the
            // direction + product and the fused update + first residual (FP64 forms), on
            // the PCG's scratch vectors with every lane active
            const TuneKey key{0, L.nx, L.ny, L.nz, B};
            int32_t zc_t = 0;
            {
                std::lock_guard<std::mutex> lk(g_tune_mu);
                auto it = g_tune.find(key);
                if (it != g_tune.end()) zc_t = it->second;
            }
            if (!zc_t) {
                MgScal* sc_t = nullptr;
                QPAT_TRY(dalloc(c, &sc_t, B));
                std::vector<MgScal> hs(B);
                for (auto& h : hs) {
                    std::memset(&h, 0, sizeof h);
                    h.active = 1;
                    h.alpha = 0.5;
                    h.beta = 0.5;   // nonzero: the direction kernel reads the old direction
                }
                QPAT_HIP(c, hipMemcpyAsync(sc_t, hs.data(), B * sizeof(MgScal), hipMemcpyHostToDevice, c->stream));
                for (double* v : {M.pa, M.pb, M.pq, M.pr, M.pr2})
                    QPAT_HIP(c, hipMemsetAsync(v, 0, L.N * B * sizeof(double), c->stream));
                const std::vector<int64_t> cands = chunk_candidates(L.nz, tx * ty, conc, false);
                std::vector<float> cms(cands.size(), 0.f);
                for (int round = 0; round < kTuneRounds; ++round)
                for (size_t ci = 0; ci < cands.size(); ++ci) {
                    set_zc(cands[ci]);
                    TileArgs g{};
                    g.nx = L.nx;
                    g.ny = L.ny;
                    g.nz = L.nz;
                    g.tiles_x = t.tiles_x;
                    g.tiles_y = t.tiles_y;
                    g.zc = t.zc;
                    g.items = t.items;
                    g.ld = B;
                    g.col = 0;
                    g.U = L.U;
                    g.dinv = L.dinv;
                    g.w = M.w;
                    g.parts = M.parts;
                    g.sc = sc_t;
                    TileArgs gd = g, gu = g;
                    gd.in = M.pa;    // z
                    gd.in2 = M.pb;   // old direction
                    gd.out = M.pq;   // q
                    gd.out2 = M.pr;  // new direction
                    gu.in = M.pr;    // r
                    gu.in2 = M.pq;   // q
                    gu.out = M.lv[0].r;
                    gu.out2 = M.pr2;
                    gu.x3 = M.pa;
                    gu.p3 = M.pb;
                    const dim3 grid(t.blocks);
                    float ms_d = 0.f, ms_u = 0.f;
                    QPAT_TRY(time_launches(c, [&] {
                        hipLaunchKernelGGL((k_mg_tile<kTDirSpmv, B>), grid, dim3(kTT), MgTile<B>::LDS, c->stream, gd);
                    }, &ms_d));
                    QPAT_TRY(time_launches(c, [&] {
                        hipLaunchKernelGGL((k_mg_tile<kTUpdResid, B>), grid, dim3(kTT), MgTile<B>::LDS, c->stream, gu);
                    }, &ms_u));
                    cms[ci] = round == 0 ? ms_d + ms_u : std::min(cms[ci], ms_d + ms_u);
                }
                zc_t = static_cast<int32_t>(cands[tune_pick(cms)]);
                QPAT_TRY(dfree(c, sc_t));
                std::lock_guard<std::mutex> lk(g_tune_mu);
                g_tune.emplace(key, zc_t);
            }
            set_zc(zc_t);
            t.tuned = true;
        }
        // restrictions to levels 1, 2, ... (coarse level of at least kTile27Min nodes): the
        // same balance with (2 zc + 1) fine planes per item
        const MgLevel& C = M.lv[1];
        const void* fr = reinterpret_cast<const void*>(&k_mg_restrict_tile<B, true>);
        for (const void* f : {fr, reinterpret_cast<const void*>(&k_mg_restrict_tile<B, false>),
                              reinterpret_cast<const void*>(&k_mg_restrict_tile<B, true, true>)})
            QPAT_HIP(c, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)MgRst<B>::LDS));
        int rocc = 1;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&rocc, fr, kTT, MgRst<B>::LDS) != hipSuccess) rocc = 1;
        const int64_t rconc = (int64_t)std::max(rocc, 1) * (cus / 8);
        for (int l = 0; l + 1 < (int)M.lv.size() && l < kMgMaxLevels; ++l) {
            const MgLevel& Q = M.lv[l + 1];
            if (l > 0 && Q.N < kTile27Min) break;
            const int64_t rtx = (Q.nx + kRX - 1) / kRX, rty = (Q.ny + MgRst<B>::RY - 1) / MgRst<B>::RY;
            int64_t rbest = -1, rzc = Q.nz;
            for (int64_t nch = 1; nch <= Q.nz; ++nch) {
                const int64_t zc = (Q.nz + nch - 1) / nch;
                const int64_t items = rtx * rty * ((Q.nz + zc - 1) / zc);
                const int64_t cost = (((items + 7) / 8 + rconc - 1) / rconc) * (2 * zc + 2);
                if (rbest < 0 || cost < rbest) {
                    rbest = cost;
                    rzc = zc;
                }
            }
            TileGeo::Rst& q = t.rst[l];
            q.tx = static_cast<int32_t>(rtx);
            q.ty = static_cast<int32_t>(rty);
            q.zc = static_cast<int32_t>(rzc);
            q.items = static_cast<int32_t>(rtx * rty * ((Q.nz + rzc - 1) / rzc));
            q.blocks = static_cast<int32_t>(8 * std::min<int64_t>(rconc, (q.items + 7) / 8));
            q.on = true;
        }
        if constexpr (B == 16) {   // the fused prolongation + last sweep: the same tiles, even chunks
            if (L.Uf && L.Ufk32) {
                for (const bool f32 : {false, true}) {
                    const void* fps = f32 ? reinterpret_cast<const void*>(&k_mg_prolong_smooth<true>)
                                          : reinterpret_cast<const void*>(&k_mg_prolong_smooth<false>);
                    const size_t lds = f32 ? kPSLds<true> : kPSLds<false>;
                    QPAT_HIP(c, hipFuncSetAttribute(fps, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                    const void* fps_c = f32 ? reinterpret_cast<const void*>(&k_mg_prolong_smooth<true, true>)
                                            : reinterpret_cast<const void*>(&k_mg_prolong_smooth<false, true>);
                    QPAT_HIP(c, hipFuncSetAttribute(fps_c, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
                    int occ_ps = 1;
                    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_ps, fps, kTT, lds) != hipSuccess) occ_ps = 1;
                    const int64_t conc_ps = (int64_t)std::max(occ_ps, 1) * (cus / 8);
                    int64_t best_ps = -1, zc_ps = L.nz + (L.nz & 1);
                    for (int64_t nch = 1; nch <= L.nz; ++nch) {
                        int64_t zc = (L.nz + nch - 1) / nch;
                        zc += zc & 1;
                        const int64_t items = tx * ty * ((L.nz + zc - 1) / zc);
                        const int64_t cost = (((items + 7) / 8 + conc_ps - 1) / conc_ps) * (zc + 2);
                        if (best_ps < 0 || cost < best_ps) {
                            best_ps = cost;
                            zc_ps = zc;
                        }
                    }
                    auto set_ps = [&](int64_t zc) {
                        const int32_t items = static_cast<int32_t>(tx * ty * ((L.nz + zc - 1) / zc));
                        (f32 ? t.ps_zc32 : t.ps_zc) = static_cast<int32_t>(zc);
                        (f32 ? t.ps_items32 : t.ps_items) = items;
                        (f32 ? t.ps_blocks32 : t.ps_blocks) =
                            static_cast<int32_t>(8 * std::min<int64_t>(conc_ps, (items + 7) / 8));
                    };
                    set_ps(zc_ps);
                    (f32 ? t.ps_zc32_model : t.ps_zc_model) = static_cast<int32_t>(zc_ps);
                    if (!c->opts.autotune) continue;
                    const TuneKey key{f32 ? 2 : 1, L.nx, L.ny, L.nz, B};
                    int32_t zc_t = 0;
                    {
                        std::lock_guard<std::mutex> lk(g_tune_mu);
                        auto it = g_tune.find(key);
                        if (it != g_tune.end()) zc_t = it->second;
                    }
                    if (!zc_t) {
                        // scratch: r in pa, z in pq, lanes all active in a private scalar array
                        MgScal* sc_t = nullptr;
                        QPAT_TRY(dalloc(c, &sc_t, B));
                        std::vector<MgScal> hs(B);
                        for (auto& h : hs) {
                            std::memset(&h, 0, sizeof h);
                            h.active = 1;
                        }
                        QPAT_HIP(c, hipMemcpyAsync(sc_t, hs.data(), B * sizeof(MgScal), hipMemcpyHostToDevice, c->stream));
                        QPAT_HIP(c, hipMemsetAsync(M.pa, 0, L.N * B * sizeof(double), c->stream));
                        QPAT_HIP(c, hipMemsetAsync(C.x, 0, C.N * B * sizeof(double), c->stream));
                        const std::vector<int64_t> cands = chunk_candidates(L.nz, tx * ty, conc_ps, true);
                        std::vector<float> cms(cands.size(), 0.f);
                        for (int round = 0; round < kTuneRounds; ++round)
                        for (size_t ci = 0; ci < cands.size(); ++ci) {
                            const int64_t zc = cands[ci];
                            set_ps(zc);
                            PSArgs g;
                            g.nx = L.nx;
                            g.ny = L.ny;
                            g.nz = L.nz;
                            g.cx = C.nx;
                            g.cy = C.ny;
                            g.cz = C.nz;
                            g.tiles_x = static_cast<int32_t>(tx);
                            g.tiles_y = static_cast<int32_t>(ty);
                            g.zc = static_cast<int32_t>(zc);
                            g.items = f32 ? t.ps_items32 : t.ps_items;
                            g.Uf = L.Ufk32;
                            g.r = M.pa;
                            g.xc = C.x;
                            g.dinv = L.dinv;
                            g.w = M.w;
                            g.z = reinterpret_cast<float*>(M.pq);
                            g.parts = M.parts;
                            g.sc = sc_t;
                            const dim3 grid(f32 ? t.ps_blocks32 : t.ps_blocks);
                            float ms = 0.f;
                            QPAT_TRY(time_launches(c, [&] {
                                if (f32)
                                    hipLaunchKernelGGL(k_mg_prolong_smooth<true>, grid, dim3(kTT), kPSLds<true>, c->stream, g);
                                else
                                    hipLaunchKernelGGL(k_mg_prolong_smooth<false>, grid, dim3(kTT), kPSLds<false>, c->stream, g);
                            }, &ms));
                            cms[ci] = round == 0 ? ms : std::min(cms[ci], ms);
                        }
                        zc_t = static_cast<int32_t>(cands[tune_pick(cms)]);
                        QPAT_TRY(dfree(c, sc_t));
                        std::lock_guard<std::mutex> lk(g_tune_mu);
                        g_tune.emplace(key, zc_t);
                    }
                    set_ps(zc_t);
                }
                t.ps_on = true;
            }
        }
        if constexpr (B == 16) {   // the coarse levels' 27-point kernels
            const void* f27[6] = {reinterpret_cast<const void*>(&k_mg_tile27<kT27Resid>),
                                  reinterpret_cast<const void*>(&k_mg_tile27<kT27Smooth>),
                                  reinterpret_cast<const void*>(&k_mg_tile27<kT27Resid, true>),
                                  reinterpret_cast<const void*>(&k_mg_tile27<kT27Smooth, true>),
                                  reinterpret_cast<const void*>(&k_mg_tile27<kT27Resid, true, true>),
                                  reinterpret_cast<const void*>(&k_mg_tile27<kT27Smooth, true, true>)};
            constexpr size_t lds27 = (size_t)3 * MgTile<16>::NPF * kTT * sizeof(double);
            for (const void* f : f27)
                QPAT_HIP(c, hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds27));
            int occ27 = 1;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ27, f27[1], kTT, lds27) != hipSuccess) occ27 = 1;
            const int64_t conc27 = (int64_t)std::max(occ27, 1) * (cus / 8);
            for (int l = 1; l < (int)M.lv.size() && l < kMgMaxLevels; ++l) {
                const MgLevel& Q = M.lv[l];
                if (!Q.Uf) continue;
                const int64_t tx27 = (Q.nx + kTHX - 3) / (kTHX - 2), ty27 = (Q.ny + kTHY - 3) / (kTHY - 2);
                int64_t best27 = -1, zc27 = Q.nz;
                for (int64_t nch = 1; nch <= Q.nz; ++nch) {
                    const int64_t zc = (Q.nz + nch - 1) / nch;
                    const int64_t items = tx27 * ty27 * ((Q.nz + zc - 1) / zc);
                    const int64_t cost = (((items + 7) / 8 + conc27 - 1) / conc27) * (zc + 2);
                    if (best27 < 0 || cost < best27) {
                        best27 = cost;
                        zc27 = zc;
                    }
                }
                TileGeo::Lv27& g27 = t.t27[l];
                g27.tx = static_cast<int32_t>(tx27);
                g27.ty = static_cast<int32_t>(ty27);
                g27.zc = static_cast<int32_t>(zc27);
                g27.items = static_cast<int32_t>(tx27 * ty27 * ((Q.nz + zc27 - 1) / zc27));
                g27.blocks = static_cast<int32_t>(8 * std::min<int64_t>(conc27, (g27.items + 7) / 8));
                g27.on = true;
            }
        }
    }
    return QPAT_OK;
}

// row kind of the V-cycle's kernels on a level
inline int vkind(const MgLevel& L) { return L.vkind >= 0 ? L.vkind : L.kind; }

// the tiled path fuses the PCG update with the V-cycle's first residual
inline bool fused_update(const TileGeo& tg) { return tg.on && kMgNu == 1; }

// the V-cycle's last finest-level sweep is the fused prolongation + sweep,
// which leaves z in FP32 (16 right-hand sides, trilinear transfer: K)
template <int B>
inline bool z32_path(const MgState& M, const TileGeo& tg) {
    return B == 16 && fused_update(tg) && tg.ps_on && !M.opdep;
}

// One right-hand side per system (M_delta), walk kernels with the FP32 Kuhn
// rows and one sweep each way: the finest level's V-cycle vectors (x0, its
// residual, z) are FP32, in the first half of their FP64 arrays. Every kernel
// that touches them has that form: the PCG update's first sweep (or the first
// sweep from zero), the residual, the restriction, the prolongation into
// level 0, the last sweep (whose dot products use z as stored) and the
// direction. The PCG's own vectors (x, r, p, q) stay FP64.
template <int B>
inline bool f32v0_path(const MgState& M, const TileGeo& tg) {
    return B == 1 && M.opdep && !tg.on && kMgNu == 1 && M.lv.size() > 1 && M.lv[0].vkind == 5 &&
           M.lv[0].N * 8 < (int64_t(1) << 31);
}

// Level 1 keeps the V-cycle's vectors (x, its ping-pong partner, r, b) in FP32,
// in the first half of their FP64 arrays, where every kernel that touches them
// has that form: 16 right-hand sides, the tiled restrictions into and out of
// level 1, its tiled 27-point residual and sweep, the prolongation into it and
// the fused prolongation + last sweep above it (preconditioner work only).
template <int B>
inline bool v32_path(const MgState& M, const TileGeo& tg) {
    return z32_path<B>(M, tg) && M.lv.size() > 2 && tiled27(tg, 1) && M.lv[1].Uf27p != nullptr && tg.rst[0].on &&
           tg.rst[1].on;
}

// One V-cycle on every lane: z = V(r), r = level 0's b. The last sweep also
// leaves the partial sums r.z, sum z, sum r. On a tiled finest level with one
// sweep each way the first sweep w D^{-1} r is never stored: the residual
// kernel stages it and the prolongation recomputes it. Level 0 takes
// 2 kMgNu - 1 ping-pong sweeps (an odd number), so z ends in level 0's t.
// lo32 (mixed precision) stages the fused last sweep's x0 in FP32.
// the smoother arguments of level l
inline SmArgs level_args(const MgState& M, int l) {
    SmArgs a;
    a.L = lv_args(M.lv[l]);
    a.dinv = M.lv[l].dinv;
    a.w = M.w;
    a.nlev = static_cast<int>(M.lv.size());
    a.lev = l;
    a.nsys = M.nsys;
    a.sc = M.sc;
    return a;
}

// first_done: the PCG update already wrote the finest level's first sweep
// (k_mgp_update_first)
template <int B>
void vcycle(const MgState& M, hipStream_t st, const TileGeo& tg, hipEvent_t* ev = nullptr, const double* b0 = nullptr,
            bool resid_done = false, bool lo32 = false, bool first_done = false) {
    const int nl = static_cast<int>(M.lv.size());
    const bool fused0 = tg.on && kMgNu == 1;
    const bool v1 = v32_path<B>(M, tg);   // level 1's vectors in FP32
    const bool f0 = f32v0_path<B>(M, tg);  // level 0's vectors in FP32 (one right-hand side)
    const double* r0 = b0 ? b0 : M.lv[0].b;   // level 0's right-hand side (the PCG residual)
    std::vector<double*> xl(nl), tl(nl);
    for (int l = 0; l < nl; ++l) {
        xl[l] = M.lv[l].x;
        tl[l] = M.lv[l].t;
    }
    auto sm = [&](int l) { return level_args(M, l); };
    for (int l = 0; l < nl - 1; ++l) {
        const MgLevel& L = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        const SmArgs a = sm(l);
        const dim3 g = sgrid<B>(L.N, M.nsys);
        const double* bl = l == 0 ? r0 : L.b;
        if (l == 0 && !fused0 && !first_done && f0)
            hipLaunchKernelGGL((k_mg_first<B, float>), sys_rows(vgrid(L.N * B), B, M.nsys), dim3(kMgT), 0, st, a, r0,
                               reinterpret_cast<float*>(xl[0]));
        else if (l == 0 && !fused0 && !first_done)
            hipLaunchKernelGGL(k_mg_first<B>, sys_rows(vgrid(L.N * B), B, M.nsys), dim3(kMgT), 0, st, a, r0, xl[0]);
        for (int k = 1; k < kMgNu; ++k) {
            launch_smooth<B, false>(vkind(L), g, st, a, bl, xl[l], tl[l], nullptr);
            std::swap(xl[l], tl[l]);
        }
        if (l == 0 && ev) (void)hipEventRecord(ev[0], st);
        if (l == 0 && fused0 && resid_done)
            ;   // the PCG update produced level 0's residual (kTUpdResid)
        else if (l == 0 && fused0)
            launch_tile<kTResidFirst, B>(M, tg, st, r0, nullptr, r0, L.r, nullptr);
        else if (l == 0 && tg.on)
            launch_tile<kTResid, B>(M, tg, st, xl[0], nullptr, r0, L.r, nullptr);
        else if (B == 16 && tiled27(tg, l))
            launch_tile27<kT27Resid>(M, tg, l, st, xl[l], L.b, L.r, v1 && l == 1);
        else if (l == 0 && f0) {
            if constexpr (B == 1)
                hipLaunchKernelGGL((k_mg_resid<5, 1, float>), g, dim3(kMgT), 0, st, a, bl,
                                   reinterpret_cast<const float*>(xl[0]), reinterpret_cast<float*>(L.r));
        } else
            QPAT_MG_KIND(vkind(L), B, k_mg_resid, g, dim3(kMgT), 0, st, a, bl, xl[l], L.r);
        if (l == 0 && ev) (void)hipEventRecord(ev[1], st);
        if (tg.on && l < kMgMaxLevels && tg.rst[l].on && !M.opdep)
            launch_restrict<B>(M, tg, l, st, xl[l + 1], v1);
        else if (M.opdep && l == 0 && f0)
            hipLaunchKernelGGL((k_mg_restrict<B, true, float>), sgrid<B>(C.N, M.nsys), dim3(kMgT), 0, st, sm(l + 1),
                               L.nx, L.ny, L.nz, reinterpret_cast<const float*>(L.r), C.b, xl[l + 1], L.Wc);
        else if (M.opdep)
            hipLaunchKernelGGL((k_mg_restrict<B, true>), sgrid<B>(C.N, M.nsys), dim3(kMgT), 0, st, sm(l + 1), L.nx,
                               L.ny, L.nz, L.r, C.b, xl[l + 1], L.Wc);
        else
            hipLaunchKernelGGL((k_mg_restrict<B, false>), sgrid<B>(C.N, M.nsys), dim3(kMgT), 0, st, sm(l + 1), L.nx, L.ny,
                               L.nz, L.r, C.b, xl[l + 1], static_cast<const float*>(nullptr));
    }
    const MgLevel& K = M.lv[nl - 1];
    hipLaunchKernelGGL(k_mg_dense<B>,
                       dim3((unsigned)((K.N + kMgT / 64 - 1) / (kMgT / 64)), (unsigned)Pk<B>::BV, (unsigned)M.nsys),
                       dim3(kMgT), K.N * sizeof(TB<B>), st, K.N, M.nsys, M.ainv, K.b, xl[nl - 1], M.sc);
    for (int l = nl - 2; l >= 0; --l) {
        const MgLevel& L = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        const SmArgs a = sm(l);
        const dim3 g = sgrid<B>(L.N, M.nsys);
        const double* bl = l == 0 ? r0 : L.b;
        if (l == 0 && z32_path<B>(M, tg)) {   // prolongation fused into the last sweep (z in FP32)
            if (ev) (void)hipEventRecord(ev[2], st);
            launch_ps(M, tg, st, r0, xl[1], tl[0], lo32, v1);
            if (ev) (void)hipEventRecord(ev[3], st);
            std::swap(xl[0], tl[0]);
            continue;
        }
        if (l == 0 && fused0 && M.opdep)
            hipLaunchKernelGGL((k_mg_prolong<B, true, true>), g, dim3(kMgT), 0, st, a, C.nx, C.ny, C.nz, xl[1],
                               r0, xl[0], L.Wc);
        else if (l == 0 && fused0)
            hipLaunchKernelGGL((k_mg_prolong<B, true, false>), g, dim3(kMgT), 0, st, a, C.nx, C.ny, C.nz, xl[1], r0,
                               xl[0], static_cast<const float*>(nullptr));
        else if (M.opdep && l == 0 && f0)   // into level 0's FP32 x0
            hipLaunchKernelGGL((k_mg_prolong<B, false, true, true>), g, dim3(kMgT), 0, st, a, C.nx, C.ny, C.nz,
                               xl[l + 1], bl, xl[l], L.Wc);
        else if (M.opdep)
            hipLaunchKernelGGL((k_mg_prolong<B, false, true>), g, dim3(kMgT), 0, st, a, C.nx, C.ny, C.nz,
                               xl[l + 1], bl, xl[l], L.Wc);
        else if (l == 1 && v1)   // into level 1's FP32 x
            hipLaunchKernelGGL((k_mg_prolong<B, false, false, true>), g, dim3(kMgT), 0, st, a, C.nx, C.ny,
                               C.nz, xl[l + 1], bl, xl[l], static_cast<const float*>(nullptr));
        else
            hipLaunchKernelGGL((k_mg_prolong<B, false, false>), g, dim3(kMgT), 0, st, a, C.nx, C.ny, C.nz, xl[l + 1],
                               bl, xl[l], static_cast<const float*>(nullptr));
        for (int k = 0; k < kMgNu; ++k) {
            const bool last = l == 0 && k == kMgNu - 1;
            if (last && ev) (void)hipEventRecord(ev[2], st);
            if (last && tg.on)
                launch_tile<kTSmoothDots, B>(M, tg, st, xl[0], nullptr, r0, tl[0], nullptr);
            else if (last && f0) {
                if constexpr (B == 1)
                    hipLaunchKernelGGL((k_mg_smooth<5, 1, true, float>), g, dim3(kMgT), 0, st, a, bl,
                                       reinterpret_cast<const float*>(xl[0]), reinterpret_cast<float*>(tl[0]),
                                       M.parts);
            } else if (last)
                launch_smooth<B, true>(vkind(L), g, st, a, bl, xl[l], tl[l], M.parts);
            else if (B == 16 && tiled27(tg, l))
                launch_tile27<kT27Smooth>(M, tg, l, st, xl[l], L.b, tl[l], v1 && l == 1);
            else
                launch_smooth<B, false>(vkind(L), g, st, a, bl, xl[l], tl[l], nullptr);
            if (last && ev) (void)hipEventRecord(ev[3], st);
            std::swap(xl[l], tl[l]);
        }
    }
}

MgState*& state_of(qpat_ctx* c, Op op) { return op == Op::K ? c->mgk : c->mg; }

template <int B>
PcgMg pcg_args(qpat_ctx* c, Op op) {
    const MgState& M = *state_of(c, op);
    PcgMg a;
    a.L = lv_args(M.lv[0]);
    a.x = c->x64;
    a.r = M.pr;
    a.po = M.pa;
    a.pn = M.pb;
    a.q = M.pq;
    a.z = M.lv[0].t;   // where the V-cycle leaves z
    a.parts = M.parts;
    a.sc = M.sc;
    const double rtol = op == Op::K ? c->opts.pcg_rtol : c->opts.prior_rtol;
    a.rtol2 = rtol * rtol;
    a.maxit = c->opts.pcg_maxit;
    a.deflate = op == Op::Prior ? c->opts.prior_deflate : 0;
    a.nsys = M.nsys;
    a.nb = static_cast<int32_t>(sgrid<B>(c->N).x);
    a.nbr = static_cast<int32_t>(vgrid(c->N, kMgGrid).x);   // k_reg_rsum, k_mgp_update_first
    a.kreg = B == 1 ? M.kreg : 0;
    a.p32 = op == Op::K && c->opts.precision == 1 ? 1 : 0;
    a.reg = M.reg;
    a.ry = M.ry;
    a.rcorr = M.rcorr;
    a.ring = 0;   // solve_B turns the direction ring on for the tiled iterations
    a.slot = M.pslot;
    a.ahist = M.ahist;
    return a;
}

// the region coarse-space part of the preconditioner for the current r
// (sums_done: the PCG update already left the partial sums of Z^T r)
template <int B>
void region_solve(const MgState& M, const PcgMg& a, hipStream_t st, bool sums_done = false) {
    if (a.kreg <= 0) return;
    // each block reduces kRegMax sums: fewer, fuller blocks than the walk kernels
    if (!sums_done)
        hipLaunchKernelGGL(k_reg_rsum, sys_rows(vgrid(a.L.N, kMgGrid), B, a.nsys), dim3(kMgT), 0, st, a, M.rparts);
    hipLaunchKernelGGL(k_reg_solve, dim3(1, a.nsys), dim3(kMgT), 0, st, a, M.rparts, M.einv, M.rsize, M.ry, M.rcorr);
}

// one iteration after the first direction: direction and product, alpha,
// update, rr, V-cycle (with r.z, sum z, sum r), beta. Iterations alternate
// the two direction buffers (par); chunks of iterations have even length.
// ev (profiling): 8 events, recorded around the direction + product, the
// update, and the finest-level residual and last sweep of the V-cycle.
template <int B>
void iteration(const MgState& M, PcgMg a, const TileGeo& tg, hipStream_t st, int par, hipEvent_t* ev = nullptr) {
    if (par) std::swap(a.po, a.pn);
    const dim3 g = sgrid<B>(a.L.N, a.nsys), lanes(1, a.nsys * B);
    if (ev) (void)hipEventRecord(ev[0], st);
    const bool p32 = a.p32 && z32_path<B>(M, tg);   // mixed precision: the direction in FP32
    RingArg ring;   // the direction ring: the slots of this iteration and the one before
    if (a.ring > 0) {
        ring.slot = a.slot;
        ring.base = reinterpret_cast<const char*>(M.pring);
        ring.stride = a.L.N * B * (p32 ? 4 : 8);
        ring.n = a.ring;
    }
    double* const xu = a.ring > 0 ? nullptr : a.x;   // with the ring, x is formed later (k_mgp_ring_flush)
    if (tg.on && p32) {
        launch_tile<kTDirSpmv, B, true, true>(M, tg, st, a.z, a.po, nullptr, a.q, a.pn, nullptr, nullptr, ring);
    } else if (tg.on && z32_path<B>(M, tg)) {   // z from the fused prolongation + last sweep, FP32
        launch_tile<kTDirSpmv, B, true>(M, tg, st, a.z, a.po, nullptr, a.q, a.pn, nullptr, nullptr, ring);
    } else if (tg.on) {
        launch_tile<kTDirSpmv, B>(M, tg, st, a.z, a.po, nullptr, a.q, a.pn, nullptr, nullptr, ring);
    } else {
        if (f32v0_path<B>(M, tg))   // z in FP32
            hipLaunchKernelGGL((k_mgp_dir<B, true>), g, dim3(kMgT), 0, st, a);
        else
            hipLaunchKernelGGL(k_mgp_dir<B>, g, dim3(kMgT), 0, st, a);
        QPAT_MG_KIND(a.L.kind, B, k_mgp_spmv, g, dim3(kMgT), 0, st, a);
    }
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_mgp_scalars, lanes, dim3(kMgT), 0, st, a, 0);
    if (ev) (void)hipEventRecord(ev[2], st);
    const bool upd1 = B == 1 && !fused_update(tg) && M.lv.size() > 1 && a.L.N * 8 < (int64_t(1) << 31);
    if (fused_update(tg)) {   // r, x and the V-cycle's first sweep + residual in one pass; r alternates buffers
        double* r_old = par ? M.pr2 : M.pr;
        double* r_new = par ? M.pr : M.pr2;
        if (p32)
            launch_tile<kTUpdResid, B, false, true>(M, tg, st, r_old, a.q, nullptr, M.lv[0].r, r_new, xu, a.pn);
        else
            launch_tile<kTUpdResid, B>(M, tg, st, r_old, a.q, nullptr, M.lv[0].r, r_new, xu, a.pn);
        a.r = r_new;
    } else if (upd1 && f32v0_path<B>(M, tg)) {   // one right-hand side: update, first sweep (FP32), region sums
        hipLaunchKernelGGL(k_mgp_update_first<float>, sys_rows(vgrid(a.L.N, kMgGrid), B, a.nsys), dim3(kMgT), 0, st,
                           a, level_args(M, 0), reinterpret_cast<float*>(M.lv[0].x), M.rparts);
    } else if (upd1) {   // one right-hand side: update, first sweep and region sums in one pass over r
        hipLaunchKernelGGL(k_mgp_update_first<double>, sys_rows(vgrid(a.L.N, kMgGrid), B, a.nsys), dim3(kMgT), 0, st,
                           a, level_args(M, 0), M.lv[0].x, M.rparts);
    } else {
        hipLaunchKernelGGL(k_mgp_update<B>, g, dim3(kMgT), 0, st, a);
    }
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL(k_mgp_scalars, lanes, dim3(kMgT), 0, st, a, 1);
    region_solve<B>(M, a, st, upd1);
    vcycle<B>(M, st, tg, ev ? ev + 4 : nullptr, a.r, fused_update(tg), p32, upd1);
    hipLaunchKernelGGL(k_mgp_scalars, lanes, dim3(kMgT), 0, st, a, 2);
}

// true residual r = b - A x of every lane, partial r.r (write_r false, tiled path:
// the partial only)
template <int B>
void true_residual(const MgState& M, const PcgMg& a, const TileGeo& tg, const double* b, hipStream_t st,
                   bool write_r = true) {
    if (tg.on)
        launch_tile<kTTrue, B>(M, tg, st, a.x, nullptr, b, write_r ? a.r : nullptr, nullptr);
    else
        QPAT_MG_KIND(a.L.kind, B, k_mgp_true, sgrid<B>(a.L.N, a.nsys), dim3(kMgT), 0, st, a, b);
}

template <int B>
qpat_status solve_B(qpat_ctx* c, Op op, SolveStats* st, bool has_x0) {
    MgState& M = *state_of(c, op);
    hipStream_t sm = c->stream;
    const int S = M.nsys * B;
    const dim3 g = sgrid<B>(c->N, M.nsys), lanes(1, S);
    PcgMg a = pcg_args<B>(c, op);
    QPAT_TRY(tile_setup<B>(c, M));
    const TileGeo tg = M.tiles[B];
    // The tiled iterations keep their directions and alphas in a ring and form
    // x = x + sum alpha_j p_j (k_mgp_ring_flush) before x is read: the update
    // then neither reads nor writes x nor reads p.
    if (fused_update(tg)) {
        if (!M.pring) {
            const size_t n = (size_t)kRing * c->N * M.bmax;   // FP64-sized slots
            QPAT_TRY(dalloc(c, &M.pring, n));
            QPAT_TRY(dalloc(c, &M.ahist, (size_t)kRing * kMgLanes));
            QPAT_TRY(dalloc(c, &M.pslot, 1));
            // finite values in the slots of lanes that stopped (their alpha is 0)
            QPAT_HIP(c, hipMemsetAsync(M.pring, 0, n * sizeof(double), sm));
        }
        a.ring = kRing;
        a.slot = M.pslot;
        a.ahist = M.ahist;
    }
    int ring_s = 0, ring_f = 0;   // iterations launched in this solve; those already added to x
    // the one-pass start leaves x unwritten with the ring: the first formation starts from zero
    bool x_zero = a.ring > 0 && tg.on && !a.deflate && !has_x0;
    auto ring_flush = [&]() -> qpat_status {
        if (a.ring == 0 || (ring_s == ring_f && !x_zero)) return QPAT_OK;
        const int64_t n = c->N * (int64_t)B;
        const bool p32r = a.p32 && z32_path<B>(M, tg);
        const int64_t stride = n * (p32r ? 4 : 8);
        const char* base = reinterpret_cast<const char*>(M.pring);
        if (B % (p32r ? 4 : 2) != 0) return fail(c, QPAT_ERR_STATE, "multigrid: direction ring with %d right-hand sides", B);
        if (p32r)
            hipLaunchKernelGGL(k_mgp_ring_flush<float>, vgrid(n, kMgBlocks), dim3(kMgT), 0, sm, n, B, a.x, base, stride,
                               M.ahist, S, ring_f, ring_s, x_zero ? 1 : 0);
        else
            hipLaunchKernelGGL(k_mgp_ring_flush<double>, vgrid(n, kMgBlocks), dim3(kMgT), 0, sm, n, B, a.x, base, stride,
                               M.ahist, S, ring_f, ring_s, x_zero ? 1 : 0);
        ring_f = ring_s;
        x_zero = false;
        QPAT_HIP(c, hipGetLastError());
        return QPAT_OK;
    };
    if (tg.on && !a.deflate && !has_x0) {   // one pass over b
        hipLaunchKernelGGL(k_mgp_start0<B>, g, dim3(kMgT), 0, sm, a, c->b64);
        hipLaunchKernelGGL(k_mgp_init, lanes, dim3(kMgT), 0, sm, a, c->delta > 0 ? 1.0 / c->delta : 0.0);
    } else {
        hipLaunchKernelGGL(k_mgp_bstats<B>, g, dim3(kMgT), 0, sm, a, c->b64);
        hipLaunchKernelGGL(k_mgp_init, lanes, dim3(kMgT), 0, sm, a, c->delta > 0 ? 1.0 / c->delta : 0.0);
        hipLaunchKernelGGL(k_mgp_start<B>, g, dim3(kMgT), 0, sm, a, c->b64, has_x0 ? 1 : 0);
    }
    if (has_x0) {   // r = b - A x0; lanes that x0 already solves stop here
        true_residual<B>(M, a, tg, c->b64, sm);
        hipLaunchKernelGGL(k_mgp_true_fin, lanes, dim3(kMgT), 0, sm, a, 1);
    }
    QPAT_HIP(c, hipGetLastError());
    auto fetch = [&]() -> qpat_status {
        QPAT_HIP(c, hipMemcpyAsync(M.sc_host, M.sc, S * sizeof(MgScal), hipMemcpyDeviceToHost, sm));
        QPAT_HIP(c, hipStreamSynchronize(sm));
        return QPAT_OK;
    };
    auto any_active = [&]() {
        for (int i = 0; i < S; ++i)
            if (M.sc_host[i].active) return true;
        return false;
    };
    std::vector<int> reopened(S, 0);   // per lane: restarts after a failed true-residual check
    for (int restart = 0; restart < 4; ++restart) {
        QPAT_TRY(fetch());
        if (!any_active()) break;
        if (restart > 0)
            for (int i = 0; i < S; ++i) reopened[i] += M.sc_host[i].active ? 1 : 0;
        // the tiled check below stores no r (its lanes almost always stop there):
        // a lane it reopened restarts from the true residual formed here
        if (restart > 0 && tg.on) true_residual<B>(M, a, tg, c->b64, sm);
        // first direction of a run: z = V(r) (+ Z y), p = z - c
        region_solve<B>(M, a, sm);
        vcycle<B>(M, sm, tg, nullptr, nullptr, false, a.p32 != 0 && z32_path<B>(M, tg));
        hipLaunchKernelGGL(k_mgp_scalars, lanes, dim3(kMgT), 0, sm, a, 3);
        QPAT_HIP(c, hipGetLastError());
        // Iterations run in chunks of even length between host checks. The
        // first is kMgChunk0 long; later ones cover the iterations that the
        // slowest lane still needs at its contraction rate over the last
        // chunk (within [2, 16]), so few iterations run after convergence. PCG
        // converges superlinearly towards the end of a run, where that rate
        // overestimates the need: a third or later chunk is therefore kept to
        // half the iterations the run has done, which bounds the iterations
        // launched after convergence (each still costs its launches) by that
        // half, at the price of a host check more on runs that long.
        int chunk = kMgChunk0, nchunk = 0;
        std::vector<int> iters_before(S, -1), iters_start(S, 0);
        std::vector<double> rr_before(S, 0.0);
        for (;;) {
            QPAT_TRY(fetch());
            if (!any_active()) break;
            if (iters_before[0] >= 0) {
                double need = 0.0;
                for (int i = 0; i < S; ++i) {
                    const MgScal& h = M.sc_host[i];
                    if (!h.active) continue;
                    const int done_its = h.iters - iters_before[i];
                    const double target = a.rtol2 * h.bnorm2;
                    if (done_its <= 0 || !(rr_before[i] > 0.0) || !(h.rr > 0.0) || h.rr >= rr_before[i]) {
                        need = 16.0;
                        continue;
                    }
                    const double rate = std::log(h.rr / rr_before[i]) / done_its;   // < 0
                    need = std::max(need, std::log(target / h.rr) / rate);
                }
                const int n = static_cast<int>(std::ceil(need));
                chunk = std::min(16, std::max(2, n + (n & 1)));
                if (nchunk >= 2) {
                    int run_its = 0;
                    for (int i = 0; i < S; ++i) run_its = std::max(run_its, M.sc_host[i].iters - iters_start[i]);
                    const int half = run_its / 2;
                    chunk = std::min(chunk, std::max(2, half + (half & 1)));
                }
            } else {
                for (int i = 0; i < S; ++i) iters_start[i] = M.sc_host[i].iters;
            }
            ++nchunk;
            for (int i = 0; i < S; ++i) {
                iters_before[i] = M.sc_host[i].iters;
                rr_before[i] = M.sc_host[i].rr;
            }
            // the chunk writes ring slots ring_s ... ring_s + chunk - 1: those not yet in x must survive
            if (a.ring > 0 && ring_s + chunk - ring_f > kRing) QPAT_TRY(ring_flush());
            ring_s += chunk;
            const bool prof = c->prof_on;
            if (prof) {
                if (M.ev.size() < (size_t)8 * chunk) {
                    const size_t old = M.ev.size();
                    M.ev.resize((size_t)8 * chunk);
                    for (size_t e = old; e < M.ev.size(); ++e) QPAT_HIP(c, hipEventCreate(&M.ev[e]));
                }
                for (int i = 0; i < chunk; ++i) iteration<B>(M, a, tg, sm, i & 1, &M.ev[8 * i]);
                QPAT_HIP(c, hipGetLastError());
                QPAT_TRY(fetch());
                // iterations after every lane stopped do no work: count the live ones
                const int base = op == Op::K ? 4 : 8;
                for (int i = 0; i < chunk; ++i) {
                    int lanes_on = 0;
                    for (int l = 0; l < S; ++l) lanes_on += (M.sc_host[l].iters - iters_before[l]) > i;
                    if (lanes_on == 0) break;
                    for (int kk = 0; kk < 4; ++kk) {
                        if (kk == 2 && fused_update(tg)) continue;   // the update's kernel did it
                        float t = 0.f;
                        QPAT_HIP(c, hipEventElapsedTime(&t, M.ev[8 * i + 2 * kk], M.ev[8 * i + 2 * kk + 1]));
                        qpat_kstat& ks = c->prof[base + kk];
                        ks.launches += 1;
                        ks.lanes += lanes_on;
                        ks.total_ms += t;
                        ks.min_ms = ks.launches == 1 ? t : std::min(ks.min_ms, (double)t);
                        ks.max_ms = std::max(ks.max_ms, (double)t);
                    }
                }
                continue;
            }
            if (c->opts.use_graphs) {
                // the chunk as graphs of 16, 8, 4 and 2 iterations (its binary
                // digits; every chunk is even), so that a solver captures at most
                // four graphs whatever chunk lengths its right-hand sides take
                for (int len = 16; len >= 2; len /= 2) {
                    if (!(chunk & len)) continue;
                    // every by-value argument of the captured kernels that can change
                    // between runs: the region count is recomputed at each prior set-up
                    char key[128];
                    snprintf(key, sizeof key, "%d/%d/%.17g/%d/%d/%d/%d", B, len, a.rtol2, a.maxit, a.deflate, a.kreg,
                             a.p32);
                    auto it = M.graphs.find(key);
                    hipGraphExec_t ex = nullptr;
                    if (it != M.graphs.end()) {
                        ex = it->second;
                    } else {
                        if (!M.cap) QPAT_HIP(c, hipStreamCreateWithFlags(&M.cap, hipStreamNonBlocking));
                        hipGraph_t gr = nullptr;
                        QPAT_HIP(c, hipStreamBeginCapture(M.cap, hipStreamCaptureModeThreadLocal));
                        for (int i = 0; i < len; ++i) iteration<B>(M, a, tg, M.cap, i & 1);
                        QPAT_HIP(c, hipStreamEndCapture(M.cap, &gr));
                        QPAT_HIP(c, hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0));
                        QPAT_HIP(c, hipGraphDestroy(gr));
                        M.graphs[key] = ex;
                    }
                    QPAT_HIP(c, hipGraphLaunch(ex, sm));
                }
            } else {
                for (int i = 0; i < chunk; ++i) iteration<B>(M, a, tg, sm, i & 1);
            }
            QPAT_HIP(c, hipGetLastError());
        }
        // confirm on the true residual; a failed check restarts from the true residual
        QPAT_TRY(ring_flush());
        true_residual<B>(M, a, tg, c->b64, sm, !tg.on);
        hipLaunchKernelGGL(k_mgp_true_fin, lanes, dim3(kMgT), 0, sm, a, restart < 3 ? 1 : 0);
        QPAT_HIP(c, hipGetLastError());
    }
    QPAT_TRY(ring_flush());   // a run that stopped before iterating still needs its x = 0
    QPAT_TRY(fetch());
    for (int i = 0; i < S; ++i) {
        const MgScal& s = M.sc_host[i];
        if (op == Op::Prior)   // the output kernel of the prior solve adds mean(b)/delta
            QPAT_HIP(c, hipMemcpyAsync(&c->scal[i].mean, &M.sc[i].mean, sizeof(double), hipMemcpyDeviceToDevice, sm));
        const double rel = s.bnorm2 > 0 ? std::sqrt(s.rr / s.bnorm2) : 0.0;
        st->add(s.iters, rel, reopened[i], s.done != 0);
    }
    return QPAT_OK;
}

}  // namespace

static void mg_drop(qpat_ctx* c, Op op) {
    MgState*& M = state_of(c, op);
    if (!M) return;
    for (auto& kv : M->graphs) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : M->ev) (void)hipEventDestroy(e);
    if (M->cap) (void)hipStreamDestroy(M->cap);
    if (M->sc_host) (void)hipHostFree(M->sc_host);
    delete M;
    M = nullptr;
}

void mg_destroy(qpat_ctx* c) {
    mg_drop(c, Op::K);
    mg_drop(c, Op::Prior);
}

bool mg_available(const qpat_ctx* c, Op op) {
    const bool want = op == Op::K ? c->opts.pcg_precond == 1 : c->opts.prior_precond == 1;
    const double* U = op == Op::K ? c->KU64 : c->MU64;
    // 32-bit element offsets in the kernels: [N][m+1] operator rows, [N][B] vectors
    return want && c->lat.on && c->opts.operator_format == 1 && U &&
           (int64_t)(c->lat.m + 1) * c->N * 8 < (int64_t(1) << 31) && c->N * kMaxRhs < (int64_t(1) << 31);
}

bool mg_ready(qpat_ctx* c, Op op) {
    const MgState* M = state_of(c, op);
    return mg_available(c, op) && M && M->current;
}

// Region coarse space of the finest level of M (one system at a time): labels
// of the strong-coupling components, the kRegMax largest regions with at
// least kRegMin nodes (with deflation: after the largest), E = Z^T A Z (exact
// integer sums) and its inverse.
static qpat_status region_setup(qpat_ctx* c, MgState& M) {
    const MgLevel& F = M.lv[0];
    const int64_t N = F.N;
    const int M1 = F.m + 1;
    if (!M.reg) {
        QPAT_TRY(dalloc(c, &M.reg, M.nsys * N));
        QPAT_TRY(dalloc(c, &M.einv, M.nsys * kRegMax * kRegMax));
        QPAT_TRY(dalloc(c, &M.rsize, M.nsys * kRegMax));
        QPAT_TRY(dalloc(c, &M.rparts, (int64_t)M.nsys * kRegMax * kMgBlocks));
        QPAT_TRY(dalloc(c, &M.ry, M.nsys * kRegMax));
        QPAT_TRY(dalloc(c, &M.rcorr, 2 * M.nsys));
    }
    int32_t *lab = nullptr, *cnt = nullptr, *flag = nullptr, *list = nullptr, *roots = nullptr;
    unsigned long long *eint = nullptr, *amax = nullptr;
    QPAT_TRY(dalloc(c, &lab, N));
    QPAT_TRY(dalloc(c, &cnt, N));
    QPAT_TRY(dalloc(c, &flag, 2));
    QPAT_TRY(dalloc(c, &list, 2 * kRegList));
    QPAT_TRY(dalloc(c, &roots, kRegMax));
    QPAT_TRY(dalloc(c, &eint, kRegMax * kRegMax));
    QPAT_TRY(dalloc(c, &amax, 1));
    hipStream_t st = c->stream;
    const dim3 g(grid_for(N, kMgT, 4096)), b(kMgT);
    std::vector<double> einv_h(M.nsys * kRegMax * kRegMax, 0.0), size_h(M.nsys * kRegMax, 0.0);
    M.kreg = 0;
    for (int sys = 0; sys < M.nsys; ++sys) {
        LvArgs L = lv_args(F);
        L.U = F.U + sys * N * M1;
        hipLaunchKernelGGL(k_reg_init, g, b, 0, st, lab, N);
        for (int round = 0;; ++round) {
            if (round > 4096) return fail(c, QPAT_ERR_DEVICE, "region labels did not settle");
            QPAT_HIP(c, hipMemsetAsync(flag, 0, sizeof(int32_t), st));
            hipLaunchKernelGGL(k_reg_prop, g, b, 0, st, L, lab, flag);
            hipLaunchKernelGGL(k_reg_jump, g, b, 0, st, lab, N);
            hipLaunchKernelGGL(k_reg_jump, g, b, 0, st, lab, N);
            int32_t fh = 0;
            QPAT_HIP(c, hipMemcpyAsync(&fh, flag, sizeof fh, hipMemcpyDeviceToHost, st));
            QPAT_HIP(c, hipStreamSynchronize(st));
            if (!fh) break;
        }
        QPAT_HIP(c, hipMemsetAsync(cnt, 0, N * sizeof(int32_t), st));
        hipLaunchKernelGGL(k_reg_count, g, b, 0, st, lab, cnt, N);
        QPAT_HIP(c, hipMemsetAsync(flag + 1, 0, sizeof(int32_t), st));
        hipLaunchKernelGGL(k_reg_roots, g, b, 0, st, lab, cnt, N, list, flag + 1);
        int32_t nl = 0;
        QPAT_HIP(c, hipMemcpyAsync(&nl, flag + 1, sizeof nl, hipMemcpyDeviceToHost, st));
        QPAT_HIP(c, hipStreamSynchronize(st));
        nl = std::min(nl, kRegList);
        std::vector<int32_t> lh(2 * std::max(nl, 1));
        if (nl > 0)
            QPAT_HIP(c, hipMemcpyAsync(lh.data(), list, 2 * nl * sizeof(int32_t), hipMemcpyDeviceToHost, st));
        QPAT_HIP(c, hipStreamSynchronize(st));
        std::vector<std::pair<int32_t, int32_t>> cand;   // (size, root)
        for (int i = 0; i < nl; ++i) cand.push_back({lh[2 * i + 1], lh[2 * i]});
        std::sort(cand.begin(), cand.end(), [](const auto& x, const auto& y) {
            return x.first != y.first ? x.first > y.first : x.second < y.second;
        });
        // With deflation the constant vector is solved exactly; the largest
        // region's indicator is then nearly that vector, and keeping it makes
        // the coarse correction all but repeat the deflated direction (PCG
        // stagnated near rtol 1e-12 with it); the other regions span its
        // complement part anyway.
        const int skip = c->opts.prior_deflate && !cand.empty() ? 1 : 0;
        cand.erase(cand.begin(), cand.begin() + skip);
        int k = std::min<int>(kRegMax, static_cast<int>(cand.size()));
        int32_t rt[kRegMax] = {};
        for (int j = 0; j < k; ++j) rt[j] = cand[j].second;
        QPAT_HIP(c, hipMemcpyAsync(roots, rt, sizeof rt, hipMemcpyHostToDevice, st));
        hipLaunchKernelGGL(k_reg_assign, g, b, 0, st, lab, N, k, roots, M.reg + sys * N);
        // E in fixed point: every sum of |contributions| stays below 2^62
        QPAT_HIP(c, hipMemsetAsync(amax, 0, sizeof(unsigned long long), st));
        hipLaunchKernelGGL(k_reg_absmax, g, b, 0, st, L.U, N * M1, amax);
        unsigned long long ab = 0;
        QPAT_HIP(c, hipMemcpyAsync(&ab, amax, sizeof ab, hipMemcpyDeviceToHost, st));
        QPAT_HIP(c, hipStreamSynchronize(st));
        double maxabs;
        std::memcpy(&maxabs, &ab, sizeof maxabs);
        if (k > 0 && maxabs > 0.0 && std::isfinite(maxabs)) {
            const double bound = static_cast<double>(N) * (2 * F.m + 1) * maxabs;
            const double scale = std::ldexp(1.0, static_cast<int>(std::floor(62.0 - std::log2(bound))));
            QPAT_HIP(c, hipMemsetAsync(eint, 0, kRegMax * kRegMax * sizeof(unsigned long long), st));
            hipLaunchKernelGGL(k_reg_e, g, b, 0, st, L, M.reg + sys * N, scale, eint);
            std::vector<unsigned long long> eh(kRegMax * kRegMax);
            QPAT_HIP(c, hipMemcpyAsync(eh.data(), eint, eh.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                       st));
            QPAT_HIP(c, hipStreamSynchronize(st));
            std::vector<double> E((size_t)k * k);
            for (int i = 0; i < k; ++i)
                for (int j = 0; j < k; ++j)
                    E[(size_t)i * k + j] = static_cast<double>(static_cast<long long>(eh[i * kRegMax + j])) / scale;
            if (!spd_inverse(E, k)) k = 0;   // not positive definite in fixed point: no region space
            for (int i = 0; i < k; ++i) {
                size_h[sys * kRegMax + i] = cand[i].first;
                for (int j = 0; j < k; ++j) einv_h[(sys * kRegMax + i) * kRegMax + j] = E[(size_t)i * k + j];
            }
        } else {
            k = 0;
        }
        if (k == 0) hipLaunchKernelGGL(k_reg_assign, g, b, 0, st, lab, N, 0, roots, M.reg + sys * N);
        M.nreg[sys] = k;
        M.kreg = std::max(M.kreg, k);
    }
    QPAT_HIP(c, hipMemcpyAsync(M.einv, einv_h.data(), einv_h.size() * sizeof(double), hipMemcpyHostToDevice, st));
    QPAT_HIP(c, hipMemcpyAsync(M.rsize, size_h.data(), size_h.size() * sizeof(double), hipMemcpyHostToDevice, st));
    QPAT_HIP(c, hipGetLastError());
    QPAT_HIP(c, hipStreamSynchronize(st));
    for (void* p : {(void*)lab, (void*)cnt, (void*)flag, (void*)list, (void*)roots, (void*)eint, (void*)amax})
        QPAT_TRY(dfree(c, p));
    return QPAT_OK;
}

// One step of the symmetric sweep operator (Gauss-Jordan elimination without
// pivoting) on each system's [n][n] matrix, pivot k, from S to T:
//   T_kk = -1/d, T_ik = S_ik/d, T_kj = S_kj/d, T_ij = S_ij - S_ik S_kj/d,  d = S_kk.
// Sweeping every pivot of an SPD matrix turns it into minus its inverse, and
// each pivot d is then a Schur-complement diagonal, so positive; the last step
// flips the sign. A pivot that is not positive sets bad[sys].
__global__ __launch_bounds__(kMgT) void k_sweep(const double* __restrict__ S, double* __restrict__ T, int n, int k,
                                                int* __restrict__ bad) {
    const int sys = blockIdx.y;
    const int64_t nn = (int64_t)n * n;
    const int64_t e = blockIdx.x * (int64_t)kMgT + threadIdx.x;
    if (e >= nn) return;
    const double* s = S + sys * nn;
    const int i = static_cast<int>(e / n), j = static_cast<int>(e % n);
    const double d = s[(int64_t)k * n + k];
    const double sg = k == n - 1 ? -1.0 : 1.0;
    double v;
    if (i == k && j == k) {
        if (!(d > 0.0) || !std::isfinite(d)) bad[sys] = 1;
        v = -1.0 / d;
    } else if (i == k) {
        v = s[e] / d;
    } else if (j == k) {
        v = s[e] / d;
    } else {
        v = s[e] - s[(int64_t)i * n + k] * s[(int64_t)k * n + j] / d;
    }
    T[sys * nn + e] = sg * v;
}

// In-place inverse of each system's SPD [n][n] matrix in M.ainv on the GPU by
// n sweep steps between M.ainv and a scratch copy (no pivoting: the matrix is
// SPD), with a check of every pivot.
qpat_status dense_spd_inverse(qpat_ctx* c, MgState& M, int n, const char* what) {
    const int64_t nn = (int64_t)n * n;
    double* tmp = nullptr;
    int* bad = nullptr;
    QPAT_TRY(dalloc(c, &tmp, M.nsys * nn));
    QPAT_TRY(dalloc(c, &bad, M.nsys));
    QPAT_HIP(c, hipMemsetAsync(bad, 0, M.nsys * sizeof(int), c->stream));
    const dim3 g((unsigned)((nn + kMgT - 1) / kMgT), (unsigned)M.nsys);
    double* src = M.ainv;
    double* dst = tmp;
    for (int k = 0; k < n; ++k) {
        hipLaunchKernelGGL(k_sweep, g, dim3(kMgT), 0, c->stream, src, dst, n, k, bad);
        std::swap(src, dst);
    }
    QPAT_HIP(c, hipGetLastError());
    if (src != M.ainv)
        QPAT_HIP(c, hipMemcpyAsync(M.ainv, src, M.nsys * nn * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
    std::vector<int> bad_h(M.nsys, 0);
    QPAT_HIP(c, hipMemcpyAsync(bad_h.data(), bad, M.nsys * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    QPAT_TRY(dfree(c, tmp));
    QPAT_TRY(dfree(c, bad));
    for (int sys = 0; sys < M.nsys; ++sys)
        if (bad_h[sys]) return fail(c, QPAT_ERR_ARG, "multigrid: coarsest %s is not positive definite", what);
    return QPAT_OK;
}

// Hierarchy for the current operator (after its assembly and stencil form).
// Called after every assembly: when the options turn multigrid off, an older
// hierarchy is marked stale so that turning it on again cannot pick it up.
qpat_status mg_setup(qpat_ctx* c, Op op) {
    MgState*& Mp = state_of(c, op);
    if (Mp) Mp->current = false;
    if (!mg_available(c, op)) return QPAT_OK;
    const int nsys = op == Op::K ? 1 : 2;
    if (!Mp) {
        Mp = new MgState();
        MgState& M = *Mp;
        M.nsys = nsys;
        M.bmax = op == Op::K ? kMaxRhs : 1;
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
        // stop at the first coarse level small enough for a dense inverse (the
        // levels below it cost a launch each for almost no work)
        while (std::max(M.lv.back().nx, std::max(M.lv.back().ny, M.lv.back().nz)) > kMgCoarse &&
               !(M.lv.size() >= 2 && M.lv.back().N <= kMgDenseK)) {
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
        if (Nc > (op == Op::K ? kMgDenseK : 4096) || nl < 2) {   // no useful hierarchy: keep Jacobi-PCG
            mg_drop(c, op);
            return QPAT_OK;
        }
        const int64_t V = (int64_t)nsys * M.bmax;
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
                QPAT_TRY(dalloc(c, &L.U, nsys * L.N * 14));
                QPAT_TRY(dalloc(c, &L.b, V * L.N));
            }
            QPAT_TRY(dalloc(c, &L.dinv, nsys * L.N));
            QPAT_TRY(dalloc(c, &L.x, V * L.N));
            QPAT_TRY(dalloc(c, &L.t, V * L.N));
            QPAT_TRY(dalloc(c, &L.r, V * L.N));
            if (op == Op::Prior && l + 1 < nl) {
                if (WPack{L.nx, L.ny, L.nz}.size() >= (int64_t(1) << 31))
                    return fail(c, QPAT_ERR_ARG, "multigrid: lattice %d x %d x %d too large for the prior's transfers",
                                L.nx, L.ny, L.nz);
                QPAT_TRY(dalloc(c, &L.W, nsys * L.N * 8));
                QPAT_TRY(dalloc(c, &L.Wc, nsys * WPack{L.nx, L.ny, L.nz}.size()));
            }
            if (op == Op::Prior && l == 0 && L.kind == 1) {   // entry-major upper rows (kind 3) and in FP32 (kind 5)
                QPAT_TRY(dalloc(c, &L.Uf, nsys * L.N * kUpRow));
                QPAT_TRY(dalloc(c, &L.Uf32, nsys * L.N * kUpRow));
            }
            if (op == Op::K && l == 0 && L.kind == 1 && M.bmax == 16 && nl > 1 &&
                L.N * kFullRow * (int64_t)sizeof(double) < (int64_t(1) << 31)) {   // node-major, for k_mg_prolong_smooth
                QPAT_TRY(dalloc(c, &L.Uf, nsys * L.N * kFullRow));
                QPAT_TRY(dalloc(c, &L.Ufk32, nsys * L.N * kFullRow));
            }
            if (op == Op::K && l >= 1 && l < kMgMaxLevels && M.bmax == 16 && M.lv[0].kind == 1 &&
                L.N >= kTile27Min && L.N * kRow27 * (int64_t)sizeof(double) < (int64_t(1) << 31)) {
                QPAT_TRY(dalloc(c, &L.Uf, nsys * L.N * kRow27));
                QPAT_TRY(dalloc(c, &L.Uf27p, nsys * L.N * kRow27));
            }
            if (op == Op::Prior && l >= 1 && l + 1 < nl && L.N >= kRow27Min) {   // entry-major rows (kind 4)
                QPAT_TRY(dalloc(c, &L.Uf, nsys * L.N * 27));
                QPAT_TRY(dalloc(c, &L.Uf32, nsys * L.N * 27));   // and in FP32 for the V-cycle (kind 6)
            }
        }
        QPAT_TRY(dalloc(c, &M.w, nsys * nl));
        QPAT_TRY(dalloc(c, &M.gmax, nsys * nl));
        QPAT_TRY(dalloc(c, &M.ainv, nsys * Nc * Nc));
        QPAT_TRY(dalloc(c, &M.pr, V * c->N));
        QPAT_TRY(dalloc(c, &M.pr2, V * c->N));
        QPAT_TRY(dalloc(c, &M.pa, V * c->N));
        QPAT_TRY(dalloc(c, &M.pb, V * c->N));
        QPAT_TRY(dalloc(c, &M.pq, V * c->N));
        QPAT_TRY(dalloc(c, &M.parts, (int64_t)kMgLanes * 4 * kMgBlocks));
        QPAT_TRY(dalloc(c, &M.sc, kMgLanes));
        QPAT_HIP(c, hipMemsetAsync(M.sc, 0, kMgLanes * sizeof(MgScal), c->stream));
        QPAT_HIP(c, hipHostMalloc((void**)&M.sc_host, kMgLanes * sizeof(MgScal), hipHostMallocDefault));
        M.lv[0].b = M.pr;   // the V-cycle acts on the PCG residual
    }
    MgState& M = *Mp;
    const int nl = static_cast<int>(M.lv.size());
    M.lv[0].U = op == Op::K ? c->KU64 : c->MU64;
    M.opdep = op == Op::Prior;
    if (M.lv[0].Uf) {   // M_delta's walk kernels (upper rows), K's fused prolongation + sweep (whole rows)
        M.lv[0].kind = 1;
        if (op == Op::K)
            hipLaunchKernelGGL(k_mg_fullrows<false>, dim3(grid_for(M.lv[0].N, kMgT, 4096), nsys), dim3(kMgT), 0,
                               c->stream, lv_args(M.lv[0]), M.lv[0].Uf);
        else
            hipLaunchKernelGGL(k_mg_fullrows<true>, dim3(grid_for(M.lv[0].N, kMgT, 4096), nsys), dim3(kMgT), 0,
                               c->stream, lv_args(M.lv[0]), M.lv[0].Uf);
        if (M.lv[0].Uf32)
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nsys * M.lv[0].N * kUpRow, kMgT, 4096)), dim3(kMgT), 0,
                               c->stream, M.lv[0].Uf, M.lv[0].Uf32, nsys * M.lv[0].N * kUpRow);
        if (M.lv[0].Ufk32)
            hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nsys * M.lv[0].N * kFullRow, kMgT, 4096)), dim3(kMgT), 0,
                               c->stream, M.lv[0].Uf, M.lv[0].Ufk32, nsys * M.lv[0].N * kFullRow);
    }
    for (int l = 0; l + 1 < nl; ++l) {
        const MgLevel& F = M.lv[l];
        const MgLevel& C = M.lv[l + 1];
        if (M.opdep) {   // prolongation weights from this level's operator, by parity class
            const dim3 g(grid_for(F.N, kMgT, 4096), nsys);
            hipLaunchKernelGGL(k_mg_pweights<0>, g, dim3(kMgT), 0, c->stream, lv_args(F), F.W);
            hipLaunchKernelGGL(k_mg_pweights<1>, g, dim3(kMgT), 0, c->stream, lv_args(F), F.W);
            hipLaunchKernelGGL(k_mg_pweights<2>, g, dim3(kMgT), 0, c->stream, lv_args(F), F.W);
            hipLaunchKernelGGL(k_mg_pweights<3>, g, dim3(kMgT), 0, c->stream, lv_args(F), F.W);
            // the transfers read the weights in FP32, packed; the Galerkin product
            // below uses the same rounded values, so A_c = P^T A P holds for the P applied
            hipLaunchKernelGGL(k_mg_wpack, g, dim3(kMgT), 0, c->stream, lv_args(F), F.W, F.Wc);
        }
        hipLaunchKernelGGL(k_mg_rap, dim3((unsigned)((C.N + kMgT - 1) / kMgT), nsys), dim3(kMgT), 0, c->stream,
                           lv_args(F), M.opdep ? F.W : nullptr, C.U, C.nx, C.ny, C.nz);
    }
    for (int l = 1; l < nl; ++l)
        if (M.lv[l].Uf && op == Op::K) {
            hipLaunchKernelGGL(k_mg_fullrows27<false>, dim3(grid_for(M.lv[l].N, kMgT, 4096), nsys), dim3(kMgT), 0,
                               c->stream, lv_args(M.lv[l]), M.lv[l].Uf);
            if (M.lv[l].Uf27p)
                hipLaunchKernelGGL(k_pairs27, dim3(grid_for(nsys * M.lv[l].N * 16, kMgT, 4096)), dim3(kMgT), 0,
                                   c->stream, nsys * M.lv[l].N, M.lv[l].Uf, M.lv[l].Uf27p);
        } else if (M.lv[l].Uf) {
            hipLaunchKernelGGL(k_mg_fullrows27<true>, dim3(grid_for(M.lv[l].N, kMgT, 4096), nsys), dim3(kMgT), 0,
                               c->stream, lv_args(M.lv[l]), M.lv[l].Uf);
            if (M.lv[l].Uf32)
                hipLaunchKernelGGL(k_to_f32, dim3(grid_for(nsys * M.lv[l].N * 27, kMgT, 4096)), dim3(kMgT), 0,
                                   c->stream, M.lv[l].Uf, M.lv[l].Uf32, nsys * M.lv[l].N * 27);
        }
    QPAT_HIP(c, hipMemsetAsync(M.gmax, 0, nsys * nl * sizeof(uint64_t), c->stream));
    for (int l = 0; l < nl; ++l)
        hipLaunchKernelGGL(k_mg_diag, dim3(grid_for(M.lv[l].N, kMgT, kMgBlocks), nsys), dim3(kMgT), 0, c->stream,
                           lv_args(M.lv[l]), M.lv[l].dinv, M.gmax, nl, l);
    QPAT_HIP(c, hipGetLastError());
    std::vector<uint64_t> gm(nsys * nl);
    QPAT_HIP(c, hipMemcpyAsync(gm.data(), M.gmax, gm.size() * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream));
    // coarsest operator to the host for its dense inverse
    const MgLevel& K = M.lv[nl - 1];
    std::vector<double> Uk(nsys * K.N * (K.m + 1));
    QPAT_HIP(c, hipMemcpyAsync(Uk.data(), K.U, Uk.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    int32_t tabk[4 * 13];
    QPAT_HIP(c, hipMemcpyAsync(tabk, K.tab, sizeof(int32_t) * 4 * K.m, hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    const char* what = op == Op::K ? "K" : "M_delta";
    std::vector<double> w(nsys * nl);
    for (int i = 0; i < nsys * nl; ++i) {
        double g;
        std::memcpy(&g, &gm[i], sizeof g);
        if (!(g > 0.0) || !std::isfinite(g)) return fail(c, QPAT_ERR_ARG, "multigrid: non-positive diagonal in %s", what);
        // finest level, coarse levels; M_delta's (strongly varying diffusivity)
        // take larger weights, still below 2 / g so that the cycle stays SPD
        if (op == Op::Prior)
            w[i] = (i % nl == 0 ? 7.0 / 4.0 : 39.0 / 20.0) / g;
        else
            w[i] = (i % nl == 0 ? 8.0 / 5.0 : 19.0 / 10.0) / g;
    }
    QPAT_HIP(c, hipMemcpyAsync(M.w, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    const int n = static_cast<int>(K.N), M1 = K.m + 1;
    const bool on_gpu = n > kMgHostDense;
    std::vector<double> inv(nsys * (size_t)n * n);
    for (int sys = 0; sys < nsys; ++sys) {
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
        if (!on_gpu && !spd_inverse(A, n))
            return fail(c, QPAT_ERR_ARG, "multigrid: coarsest %s is not positive definite", what);
        std::copy(A.begin(), A.end(), inv.begin() + (size_t)sys * n * n);
    }
    QPAT_HIP(c, hipMemcpyAsync(M.ainv, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (on_gpu) QPAT_TRY(dense_spd_inverse(c, M, n, what));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    if (op == Op::Prior) QPAT_TRY(region_setup(c, M));
    if (M.lv[0].Uf && op == Op::Prior) M.lv[0].kind = 3;
    if (M.lv[0].Uf32 && op == Op::Prior) M.lv[0].vkind = 5;   // the V-cycle's sweeps and residuals on FP32 rows
    for (int l = 1; op == Op::Prior && l < nl; ++l) {
        if (M.lv[l].Uf) M.lv[l].kind = 4;
        if (M.lv[l].Uf32) M.lv[l].vkind = 6;   // the V-cycle's sweeps and residuals on FP32 rows
    }
    M.current = true;
    return QPAT_OK;
}

// out [N][B] = scale U in, U a Kuhn stencil form [N][8] of the lattice, in
// [N][ld] (columns col ... col + B - 1), with the LDS-tiled kernel of the K
// hierarchy's finest level. false: that tiling is not available for B.
template <int B>
static qpat_status apply_B(qpat_ctx* c, const double* U, const double* in, int ld, int col, double* out,
                           double scale, bool* done) {
    *done = false;
    if constexpr (B >= 8) {
        MgState* M = state_of(c, Op::K);
        if (!M || !mg_ready(c, Op::K)) return QPAT_OK;
        QPAT_TRY(tile_setup<B>(c, *M));
        const TileGeo& t = M->tiles[B];
        if (!t.on) return QPAT_OK;
        const MgLevel& L = M->lv[0];
        if ((int64_t)L.nx * L.ny * ld * (int64_t)sizeof(double) >= (int64_t(1) << 31)) return QPAT_OK;
        TileArgs g{};
        g.nx = L.nx;
        g.ny = L.ny;
        g.nz = L.nz;
        g.tiles_x = t.tiles_x;
        g.tiles_y = t.tiles_y;
        g.zc = t.zc;
        g.items = t.items;
        g.ld = ld;
        g.col = col;
        g.scale = scale;
        g.U = U;
        g.in = in;
        g.out = out;
        hipLaunchKernelGGL((k_mg_tile<kTApply, B>), dim3(t.blocks), dim3(kTT), MgTile<B>::LDS, c->stream, g);
        QPAT_HIP(c, hipGetLastError());
        *done = true;
    }
    return QPAT_OK;
}

qpat_status mg_tile_schedule(const qpat_ctx* c, int B, int32_t out[8]) {
    const MgState* M = state_of(const_cast<qpat_ctx*>(c), Op::K);
    if (!M) return QPAT_ERR_STATE;
    const auto it = M->tiles.find(B);
    if (it == M->tiles.end() || !it->second.ready) return QPAT_ERR_STATE;
    const TileGeo& t = it->second;
    out[0] = t.on ? 1 : 0;
    out[1] = t.on ? t.zc : 0;
    out[2] = t.on ? t.zc_model : 0;
    out[3] = t.ps_on ? t.ps_zc : 0;
    out[4] = t.ps_on ? t.ps_zc_model : 0;
    out[5] = t.ps_on ? t.ps_zc32 : 0;
    out[6] = t.ps_on ? t.ps_zc32_model : 0;
    out[7] = t.tuned ? 1 : 0;
    return QPAT_OK;
}

qpat_status mg_stencil_apply(qpat_ctx* c, int B, const double* U, const double* in, int ld, int col, double* out,
                             double scale, bool* done) {
    switch (B) {
        case 8: return apply_B<8>(c, U, in, ld, col, out, scale, done);
        case 16: return apply_B<16>(c, U, in, ld, col, out, scale, done);
        default: *done = false; return QPAT_OK;
    }
}

// A x = b with the multigrid-preconditioned PCG: b in c->b64 ([nsys][N][B],
// overwritten by its deflated form), x in c->x64 (has_x0: it holds the
// start); for M_delta c->scal[sys].mean receives mean(b)/delta.
qpat_status mg_solve(qpat_ctx* c, Op op, int B, SolveStats* st, bool has_x0) {
    if (B > state_of(c, op)->bmax) return fail(c, QPAT_ERR_ARG, "multigrid: block of %d right-hand sides", B);
    switch (B) {
        case 1: return solve_B<1>(c, op, st, has_x0);
        case 2: return solve_B<2>(c, op, st, has_x0);
        case 4: return solve_B<4>(c, op, st, has_x0);
        case 8: return solve_B<8>(c, op, st, has_x0);
        case 16: return solve_B<16>(c, op, st, has_x0);
        default: return fail(c, QPAT_ERR_ARG, "multigrid: block size %d not supported", B);
    }
}

}  // namespace qpat
