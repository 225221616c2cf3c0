// Block Jacobi-PCG on the sliced-ELL operator, B independent right-hand sides
// interleaved [N][B] per system, nsys systems sharing one pattern.
//
// Every K^{-1} (Appendix: "operate with the inverse of the FEM system
// matrix") and every M_delta^{-1} (Sec. 4, one per LSQR round) of the path
// goes through this engine. Stopping rule: ||b - A x||_2 <= rtol ||b||_2 on
// the FP64 true residual.
//
// One iteration is two kernels:
//   dir_spmv : p <- D^{-1} r - c + beta p (recomputed on the fly for every
//              gathered neighbour, p ping-pongs between two buffers),
//              q = A p, partial p.q; the last block to finish reduces the
//              partials in fixed order and sets alpha = r.z / p.q.
//   update   : x += alpha p, r -= alpha q, partial r.D^{-1}r and r.r (and
//              the deflation sums); the last block sets beta and flags.
// All scalars stay on the device; the host reads them once per chunk of
// iterations to schedule FP64 true-residual recomputations (reliable updates
// in mixed precision, confirmation of convergence in both modes).
// Deflation (prior only): M_delta has the exact eigenpair (delta, 1) per
// block; the mean of the solution is mean(b)/delta and PCG runs on the
// complement of the constants with the projected preconditioner
// z = D^{-1} r - mean(D^{-1} r).
#include <cmath>

#include "qpat_internal.h"

namespace qpat {
namespace {

constexpr int kUnroll = 16;   // neighbours gathered per row before the arithmetic
constexpr int kMaxBlocks = 2048;  // blocks per system (partial-sum buffer: 5 x kMaxSys x kMaxBlocks)

template <typename T>
struct PcgArgs {
    Sell s;
    int64_t N;
    int32_t nsys;
    int32_t gs;          // blocks per system (multiple of 8)
    int32_t rpb;         // rows per block (multiple of 64)
    const T* vals;       // [nsys][len]
    const T* dinv;       // [nsys][N]
    const double* vals64;
    const double* dinv64;
    T* r;                // [nsys][N][B]
    T* pa;
    T* pb;
    T* q;
    T* x;                // low-precision iterate (FP64 mode: x64 itself)
    double* x64;
    double* b64;
    PcgScal* sc;
    PcgShared* sh;
    double* partials;
    double rtol2;
    int32_t maxit;
    uint32_t mask;       // lanes of a true-residual recomputation
    double inv_delta;
    // FP64 stencil form for the true residual (null: sliced ELL)
    const double* u64;   // [nsys][N][m+1]
    const int4* tab;     // [m] dx, dy, dz, dx + nx (dy + ny dz)
    int32_t nx, ny, nz, m;
};

// Tiling of the stencil direction+SpMV kernel (lattice meshes). A work item
// is a tile of tx x ty lattice columns over a chunk of zc planes; a block
// sweeps the chunk plane by plane with the direction vector of three planes
// (plus a one-node halo) in LDS.
template <typename T>
struct StArgs {
    bool on;
    bool kuhn;           // the Kuhn offsets: the kernel specialised on them
    int32_t nx, ny, nz, m;
    const int4* tab;     // [m] upper offsets: dx, dy, dz, dx + nx (dy + ny dz)
    const T* U;          // [nsys][N][m+1]
    int32_t hx, hy;      // halo'd tile: (hx - 2) x (hy - 2) output columns
    int32_t tiles_x, tiles_y, zc, items;
};

__device__ __forceinline__ double ld_acq(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// XCD-aware block -> row-range map: consecutive hardware blocks go to
// different XCDs, so give each XCD a contiguous band of rows.
__device__ __forceinline__ void block_rows(int32_t gs, int32_t rpb, int64_t N, int32_t& sys, int64_t& r0,
                                           int64_t& r1) {
    int32_t bx = blockIdx.x;
    sys = bx / gs;
    int32_t local = bx % gs;
    int32_t lb = (local & 7) * (gs >> 3) + (local >> 3);
    r0 = (int64_t)lb * rpb;
    r1 = r0 + rpb;
    if (r1 > N) r1 = N;
}

// sum over threads with equal (tid % B); result valid in threads tid < B
template <int B>
__device__ __forceinline__ double block_sum(double v, double* sm) {
#pragma unroll
    for (int off = 32; off >= B; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < B) sm[wave * B + lane] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < B) t = sm[threadIdx.x] + sm[B + threadIdx.x] + sm[2 * B + threadIdx.x] + sm[3 * B + threadIdx.x];
    __syncthreads();
    return t;
}

__device__ __forceinline__ void write_partial(double* partials, int v, int gs, double val) {
    const int32_t local = blockIdx.x % gs;
    partials[(int64_t)v * gs + local] = val;
}

__device__ void count_active(PcgScal* sc, PcgShared* sh, int S) {
    if (threadIdx.x == 0) {
        int n = 0;
        for (int i = 0; i < S; ++i) n += sc[i].active;
        sh->n_active = n;
    }
}

// ---------------------------------------------------------------- iteration
template <typename T, int B, bool DEFL>
__global__ __launch_bounds__(kThreads) void k_dir_spmv(PcgArgs<T> a) {
    __shared__ double sm[4 * kMaxRhs];
    if (a.sh->n_active == 0) return;
    int32_t sys;
    int64_t r0, r1;
    block_rows(a.gs, a.rpb, a.N, sys, r0, r1);
    const int k = threadIdx.x % B;
    const int sidx = sys * B + k;
    const int par = a.sh->parity;
    const T* __restrict__ pold = par ? a.pb : a.pa;
    T* __restrict__ pnew = par ? a.pa : a.pb;
    const PcgScal scl = a.sc[sidx];
    const bool act = scl.active != 0;
    const T beta = static_cast<T>(scl.beta);
    const T cc = DEFL ? static_cast<T>(scl.c) : T(0);
    const T* __restrict__ vals = a.vals + (int64_t)sys * a.s.len;
    const T* __restrict__ dinv = a.dinv + (int64_t)sys * a.N;
    const T* __restrict__ r = a.r + (int64_t)sys * a.N * B;
    const T* __restrict__ po = pold + (int64_t)sys * a.N * B;
    T* __restrict__ pn = pnew + (int64_t)sys * a.N * B;
    T* __restrict__ q = a.q + (int64_t)sys * a.N * B;
    const int32_t* __restrict__ cols = a.s.cols;
    double acc = 0.0;
    for (int64_t row = r0 + threadIdx.x / B; row < r1; row += kThreads / B) {
        const int64_t idx = row * B + k;
        if (act) {
            const int32_t base = a.s.slice_ptr[row / kSlice] + static_cast<int32_t>(row % kSlice);
            const int32_t n = a.s.rowlen[row];
            // all column indices and values first, then all gathers: two memory
            // round trips per row instead of two per neighbour
            int32_t col[kUnroll];
            T av[kUnroll];
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                col[j] = j < n ? cols[base + j * kSlice] : static_cast<int32_t>(row);
                av[j] = j < n ? vals[base + j * kSlice] : T(0);
            }
            const T pi = dinv[row] * r[idx] - cc + beta * po[idx];
            T sum = T(0);
#pragma unroll
            for (int j = 0; j < kUnroll; ++j) {
                const int64_t jdx = (int64_t)col[j] * B + k;
                const T pj = dinv[col[j]] * r[jdx] - cc + beta * po[jdx];
                sum += av[j] * pj;
            }
            for (int32_t j = kUnroll; j < n; ++j) {   // rows longer than kUnroll (unstructured meshes)
                const int32_t cj = cols[base + j * kSlice];
                const int64_t jdx = (int64_t)cj * B + k;
                sum += vals[base + j * kSlice] * (dinv[cj] * r[jdx] - cc + beta * po[jdx]);
            }
            pn[idx] = pi;
            q[idx] = sum;
            acc += static_cast<double>(pi) * static_cast<double>(sum);
        } else {
            pn[idx] = po[idx];
        }
    }
    double bs = block_sum<B>(acc, sm);
    if (threadIdx.x < B) write_partial(a.partials, sys * B + threadIdx.x, a.gs, bs);
}

// Direction + SpMV on the lattice form. Same arithmetic as k_dir_spmv: the
// direction p = D^{-1} r - c + beta p_old is formed once per node (and halo
// node) as its plane enters a three-plane ring in LDS, then every output node
// of the middle plane gathers its neighbours from LDS:
//   q_i = U_0[i] p_i + sum_j ( U_j[i] p_{i+u_j} + U_j[i-u_j] p_{i-u_j} ).
// With NPU > 0 the stored diagonals of planes z-1 and z are staged in LDS as
// well (coalesced loads; B >= 8 right-hand sides share every value), else
// they are read from global memory per node. The loads of plane z+2 are in
// flight during the arithmetic of plane z. Element offsets are 32-bit (the
// lattice form is only enabled when N (m+1) and N B fit).
constexpr int kStThreads = 512;

template <int B, int NT>
__device__ __forceinline__ double block_sum_n(double v, double* sm) {
#pragma unroll
    for (int off = 32; off >= B; off >>= 1) v += __shfl_xor(v, off);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane < B) sm[wave * B + lane] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < B)
        for (int w = 0; w < NT / 64; ++w) t += sm[w * B + threadIdx.x];
    __syncthreads();
    return t;
}

// upper offsets of the Kuhn split along the (1,1,1) diagonal, in the order the
// lattice setup numbers them (ascending (dx+1) + 3 (dy+1) + 9 (dz+1))
constexpr int kKuhnM = 7;
constexpr int kKdx[kKuhnM] = {1, 0, 1, 0, 1, 0, 1};
constexpr int kKdy[kKuhnM] = {0, 1, 1, 0, 0, 1, 1};
constexpr int kKdz[kKuhnM] = {0, 0, 0, 1, 1, 1, 1};

// HXC > 0: the Kuhn offsets above and a halo'd tile width of HXC, both known
// at compile time, so every LDS offset of the gather is an immediate.
// HXC = 0: any lattice stencil (offsets from g.tab, tile width g.hx).
template <typename T, int B, bool DEFL, int NPF, int NU, int HXC>
__global__ __launch_bounds__(kStThreads, 4) void k_dir_stencil(PcgArgs<T> a, StArgs<T> g) {
    constexpr bool KUHN = HXC > 0;
    constexpr int NT = kStThreads;
    constexpr int RS = NPF * NT;   // ring slot stride (>= halo nodes x B); the tail is padding
    constexpr int US = NU * NT;    // staged-diagonal slot stride (>= halo nodes x (m+1))
    constexpr uint32_t SZ = sizeof(T);
    extern __shared__ __align__(16) unsigned char st_smem[];
    __shared__ double sm[(NT / 64) * kMaxRhs];
    if (a.sh->n_active == 0) return;
    const int32_t sys = blockIdx.x / a.gs, local = blockIdx.x % a.gs;
    const int tid = threadIdx.x;
    const int k = tid % B;
    const int par = a.sh->parity;
    const PcgScal scl = a.sc[sys * B + k];
    const bool act = scl.active != 0;
    const T beta = static_cast<T>(scl.beta);
    const T cc = DEFL ? static_cast<T>(scl.c) : T(0);
    const T alpha = static_cast<T>(scl.alpha);   // pending x += alpha p_old of the last iteration
    const int64_t N = a.N;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int m = KUHN ? kKuhnM : g.m;
    const int M1 = m + 1;
    const int hx = KUHN ? HXC : g.hx;
    const int hn = hx * g.hy, tx = hx - 2, ty = g.hy - 2;
    const int64_t nxy = (int64_t)nx * ny;
    const uint32_t pv = static_cast<uint32_t>(nxy) * B * SZ;           // bytes of one plane of a vector
    const uint32_t pu = static_cast<uint32_t>(nxy) * M1 * SZ;          // one plane of the stencil arrays
    const T* __restrict__ dinv = a.dinv + (int64_t)sys * N;
    const T* __restrict__ r = a.r + (int64_t)sys * N * B;
    const T* __restrict__ po = (par ? a.pb : a.pa) + (int64_t)sys * N * B;
    T* __restrict__ pn = (par ? a.pa : a.pb) + (int64_t)sys * N * B;
    T* __restrict__ q = a.q + (int64_t)sys * N * B;
    T* __restrict__ xv = a.x + (int64_t)sys * N * B;
    const T* __restrict__ U = g.U + (int64_t)sys * M1 * N;
    T* ring = reinterpret_cast<T*>(st_smem);          // [3][RS]: [halo node][B]
    T* ust = ring + 3 * RS;                           // [3][US]: [halo node][m+1]
    // a plane's buffer resource; planes outside the lattice have no records,
    // so their loads return 0 and their stores are dropped
    auto plane = [&](const T* base, int pl, int64_t stride, uint32_t bytes) {
        const bool in = pl >= 0 && pl < nz;
        return rsrc(base + (in ? pl * stride : 0), in ? bytes : 0u);
    };

    // LDS element index of output slot u in a ring slot (slots past the tile
    // point at an interior position; their results are not stored)
    int32_t oc0[NPF];
#pragma unroll
    for (int u = 0; u < NPF; ++u) {
        const int nl = (tid + u * NT) / B;
        oc0[u] = nl < tx * ty ? (nl / tx + 1) * hx + nl % tx + 1 : hx + 1;
    }

    T rr[NPF], pp[NPF], dd[NPF], uu[NU];
    bool fz = false;
    double acc = 0.0;

    const int32_t xcd = local & 7, slot = local >> 3, per = a.gs >> 3;
    const int32_t wx = (g.items + 7) / 8;
    const int32_t it_end = min(g.items, (xcd + 1) * wx);
    const int32_t tiles = g.tiles_x * g.tiles_y;
    for (int32_t item = xcd * wx + slot; item < it_end; item += per) {
        const int32_t ch = item / tiles, t2 = item % tiles;
        const int32_t x0 = (t2 % g.tiles_x) * tx, y0 = (t2 / g.tiles_x) * ty;
        const int32_t zb = ch * g.zc, ze = min(zb + g.zc, nz);
        // byte offsets inside a plane of this tile's slots (kOut: outside the
        // lattice or the tile -- past every resource's records)
        uint32_t fo[NPF], oo[NPF], uo[NU];
#pragma unroll
        for (int u = 0; u < NPF; ++u) {
            const int nl = (tid + u * NT) / B;
            const int gx = x0 - 1 + nl % hx, gy = y0 - 1 + nl / hx;
            const bool fin = nl < hn && gx >= 0 && gx < nx && gy >= 0 && gy < ny;
            fo[u] = fin ? (static_cast<uint32_t>(gy * nx + gx) * B + k) * SZ : kOut;
            const int ox = x0 + nl % tx, oy = y0 + nl / tx;
            const bool oin = nl < tx * ty && ox < nx && oy < ny;
            oo[u] = oin ? (static_cast<uint32_t>(oy * nx + ox) * B + k) * SZ : kOut;
        }
#pragma unroll
        for (int v = 0; v < NU; ++v) {
            const int e = tid + v * NT, nl = e / M1;
            const int gx = x0 - 1 + nl % hx, gy = y0 - 1 + nl / hx;
            uo[v] = (nl < hn && gx >= 0 && gx < nx && gy >= 0 && gy < ny)
                        ? (static_cast<uint32_t>(gy * nx + gx) * M1 + e % M1) * SZ
                        : kOut;
        }

        // loads are unconditional (the range check zeroes halo and edge slots),
        // so they issue back to back without branches
        auto fetch = [&](int pl) {
            fz = pl >= 0 && pl < nz;
            const auto br = plane(r, pl, nxy * B, pv), bp = plane(po, pl, nxy * B, pv);
            const auto bd = plane(dinv, pl, nxy, pv / B), bu = plane(U, pl, nxy * M1, pu);
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                rr[u] = bload<T>(br, fo[u]);
                pp[u] = bload<T>(bp, fo[u]);
                dd[u] = bload<T>(bd, (fo[u] - k * SZ) / B);   // kOut maps past the plane too
            }
#pragma unroll
            for (int v = 0; v < NU; ++v) uu[v] = bload<T>(bu, uo[v]);
        };
        auto store = [&](int sl) {
            T* R = ring + sl * RS;
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                const T v = dd[u] * rr[u] - cc + beta * pp[u];
                R[tid + u * NT] = (!DEFL || (fz && fo[u] != kOut)) ? v : T(0);
            }
            T* S = ust + sl * US;
#pragma unroll
            for (int v = 0; v < NU; ++v) S[tid + v * NT] = uu[v];
        };
        // plane z with ring/diagonal slots (z, z+1, z-1) = (SZ0, SP0, SL0)
        auto step = [&](int z, auto SZ0, auto SP0, auto SL0) {
            constexpr int sz = decltype(SZ0)::value, sp = decltype(SP0)::value, sl = decltype(SL0)::value;
            store(sp);
            __syncthreads();
            if (z + 1 < ze) fetch(z + 2);
            const auto bpn = plane(pn, z, nxy * B, pv), bq = plane(q, z, nxy * B, pv);
            // the deferred iterate update of the output nodes: loads issued here,
            // in flight during the arithmetic below
            // (per-lane choices go into the offsets: a descriptor must stay
            // uniform over the wavefront)
            const auto bx = plane(xv, z, nxy * B, pv);
            const auto bo = plane(po, z, nxy * B, pv);   // inactive lanes copy p
            const bool xup = alpha != T(0), pold = alpha != T(0) || !act;
            T xo[NPF], pov[NPF];
#pragma unroll
            for (int u = 0; u < NPF; ++u) {
                xo[u] = bload<T>(bx, xup ? oo[u] : kOut);
                pov[u] = bload<T>(bo, pold ? oo[u] : kOut);
            }
            if (act) {
                const T* Rz = ring + sz * RS;
                const T* Sz = ust + sz * US;
                const T* Rp = ring + sp * RS;
                const T* Rm = ring + sl * RS;
                const T* Sm = ust + sl * US;
                // q_i = U_0 p_i + sum_j U_j[i] p_{i+u_j} + U_j[i-u_j] p_{i-u_j}
                auto row = [&](int c0) {
                    T sum = Sz[c0 * M1] * Rz[c0 * B + k];
                    auto term = [&](int j, int dx, int dy, int dz) {
                        const int d = dy * hx + dx;
                        const T* Ru = dz ? Rp : Rz;
                        const T* Rl = dz ? Rm : Rz;
                        const T* Sl = dz ? Sm : Sz;
                        sum += Sz[c0 * M1 + j] * Ru[(c0 + d) * B + k] + Sl[(c0 - d) * M1 + j] * Rl[(c0 - d) * B + k];
                    };
                    if constexpr (KUHN) {
                        // byte offsets from the tile-corner neighbour (c0 - hx - 1) are all
                        // non-negative compile-time constants: LDS reads with immediate offsets
                        const char* rb = reinterpret_cast<const char*>(ring) + ((c0 - HXC - 1) * B + k) * SZ;
                        const char* ub = reinterpret_cast<const char*>(ust) + (c0 - HXC - 1) * (kKuhnM + 1) * SZ;
                        constexpr int cc = HXC + 1;
                        auto R = [&](int sl_, int at) {
                            return *reinterpret_cast<const T*>(rb + (sl_ * RS + at * B) * SZ);
                        };
                        auto S = [&](int sl_, int at, int j) {
                            return *reinterpret_cast<const T*>(ub + (sl_ * US + at * (kKuhnM + 1) + j) * SZ);
                        };
                        sum = S(sz, cc, 0) * R(sz, cc);
#pragma unroll
                        for (int j = 0; j < kKuhnM; ++j) {
                            const int d = kKdy[j] * HXC + kKdx[j];
                            const int up = kKdz[j] ? sp : sz, lo = kKdz[j] ? sl : sz;
                            sum += S(sz, cc, j + 1) * R(up, cc + d) + S(lo, cc - d, j + 1) * R(lo, cc - d);
                        }
                    } else {
#pragma unroll 1
                        for (int j = 0; j < m; ++j) {
                            const int4 t = g.tab[j];          // dx, dy, dz, dx + nx (dy + ny dz)
                            term(j + 1, t.x, t.y, t.z);
                        }
                    }
                    return sum;
                };
#pragma unroll
                for (int u = 0; u < NPF; ++u) {
                    if (tid + u * NT >= tx * ty * B) continue;   // whole waves past the tile skip
                    const T pc = Rz[oc0[u] * B + k];
                    const T sum = row(oc0[u]);
                    bstore<T>(bpn, oo[u], pc);
                    bstore<T>(bq, oo[u], sum);
                    acc += oo[u] != kOut ? static_cast<double>(pc) * static_cast<double>(sum) : 0.0;
                }
            } else {
#pragma unroll
                for (int u = 0; u < NPF; ++u) bstore<T>(bpn, oo[u], pov[u]);
            }
            // with alpha = 0 nothing is stored
#pragma unroll
            for (int u = 0; u < NPF; ++u) bstore<T>(bx, xup ? oo[u] : kOut, xo[u] + alpha * pov[u]);
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
    const double bs = block_sum_n<B, NT>(acc, sm);
    if (tid < B) write_partial(a.partials, sys * B + tid, a.gs, bs);
}

// XD: the iterate update x += alpha p is deferred to the next direction
// kernel (which reads p anyway), so this kernel only updates r
template <typename T, int B, bool DEFL, bool XD>
__global__ __launch_bounds__(kThreads) void k_update(PcgArgs<T> a) {
    __shared__ double sm[4 * kMaxRhs];
    if (a.sh->n_active == 0) return;
    int32_t sys;
    int64_t r0, r1;
    block_rows(a.gs, a.rpb, a.N, sys, r0, r1);
    const int k = threadIdx.x % B;
    const int sidx = sys * B + k;
    const int par = a.sh->parity;
    const T* __restrict__ p = (par ? a.pb : a.pa) + (int64_t)sys * a.N * B;
    const PcgScal scl = a.sc[sidx];
    const bool act = scl.active != 0;
    const T alpha = static_cast<T>(scl.alpha);
    const T* __restrict__ dinv = a.dinv + (int64_t)sys * a.N;
    T* __restrict__ r = a.r + (int64_t)sys * a.N * B;
    T* __restrict__ x = a.x + (int64_t)sys * a.N * B;
    const T* __restrict__ q = a.q + (int64_t)sys * a.N * B;
    double rz = 0.0, rr = 0.0, z1 = 0.0, r1s = 0.0;
    if (act) {
        constexpr int RS = kThreads / B;   // row stride of one pass
        int64_t row = r0 + threadIdx.x / B;
        // four rows per iteration: their loads are independent and go out together
        for (; row + 3 * RS < r1; row += 4 * RS) {
            T xv[4], pv[4], qv[4], rv[4], dv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t idx = (row + u * RS) * B + k;
                if (!XD) {
                    xv[u] = x[idx];
                    pv[u] = p[idx];
                }
                qv[u] = q[idx];
                rv[u] = r[idx];
                dv[u] = dinv[row + u * RS];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int64_t idx = (row + u * RS) * B + k;
                const T ri = rv[u] - alpha * qv[u];
                if (!XD) x[idx] = xv[u] + alpha * pv[u];
                r[idx] = ri;
                const T zi = dv[u] * ri;
                rz += static_cast<double>(ri) * static_cast<double>(zi);
                rr += static_cast<double>(ri) * static_cast<double>(ri);
                if (DEFL) {
                    z1 += static_cast<double>(zi);
                    r1s += static_cast<double>(ri);
                }
            }
        }
        for (; row < r1; row += RS) {
            const int64_t idx = row * B + k;
            const T ri = r[idx] - alpha * q[idx];
            if (!XD) x[idx] = x[idx] + alpha * p[idx];
            r[idx] = ri;
            const T zi = dinv[row] * ri;
            rz += static_cast<double>(ri) * static_cast<double>(zi);
            rr += static_cast<double>(ri) * static_cast<double>(ri);
            if (DEFL) {
                z1 += static_cast<double>(zi);
                r1s += static_cast<double>(ri);
            }
        }
    }
    constexpr int Q = DEFL ? 4 : 2;
    const int S = a.nsys * B;
    double v0 = block_sum<B>(rz, sm);
    double v1 = block_sum<B>(rr, sm);
    double v2 = 0.0, v3 = 0.0;
    if (DEFL) {
        v2 = block_sum<B>(z1, sm);
        v3 = block_sum<B>(r1s, sm);
    }
    if (threadIdx.x < B) {
        const int v = sys * B + threadIdx.x;
        write_partial(a.partials, v, a.gs, v0);
        write_partial(a.partials, S + v, a.gs, v1);
        if (DEFL) {
            write_partial(a.partials, 2 * S + v, a.gs, v2);
            write_partial(a.partials, 3 * S + v, a.gs, v3);
        }
    }
}

// ------------------------------------------------------- true residual (FP64)
// mixed precision: fold the low-precision iterate into x64 first
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_fold(PcgArgs<T> a) {
    int32_t sys;
    int64_t r0, r1;
    block_rows(a.gs, a.rpb, a.N, sys, r0, r1);
    const int k = threadIdx.x % B;
    if (!((a.mask >> (sys * B + k)) & 1u)) return;
    T* __restrict__ x = a.x + (int64_t)sys * a.N * B;
    double* __restrict__ x64 = a.x64 + (int64_t)sys * a.N * B;
    for (int64_t row = r0 + threadIdx.x / B; row < r1; row += kThreads / B) {
        const int64_t idx = row * B + k;
        x64[idx] += static_cast<double>(x[idx]);
        x[idx] = T(0);
    }
}

// deferred iterate update: x += alpha p (current direction) for every lane
// whose last update is still pending; k_alpha_done then clears alpha
template <typename T, int B>
__global__ __launch_bounds__(kThreads) void k_xflush(PcgArgs<T> a) {
    int32_t sys;
    int64_t r0, r1;
    block_rows(a.gs, a.rpb, a.N, sys, r0, r1);
    const int k = threadIdx.x % B;
    const T alpha = static_cast<T>(a.sc[sys * B + k].alpha);
    if (alpha == T(0)) return;
    const T* __restrict__ p = (a.sh->parity ? a.pb : a.pa) + (int64_t)sys * a.N * B;
    T* __restrict__ x = a.x + (int64_t)sys * a.N * B;
    for (int64_t row = r0 + threadIdx.x / B; row < r1; row += kThreads / B) {
        const int64_t idx = row * B + k;
        x[idx] += alpha * p[idx];
    }
}

__global__ void k_alpha_done(PcgScal* sc, int S) {
    if (threadIdx.x < S) sc[threadIdx.x].alpha = 0.0;
}

// r = b - A64 x64 for the masked lanes; replaces the recursive residual and
// decides convergence on it. With init = true (all lanes, x64 = 0 assumed when
// has_x0 is false) it also sets up the run.
template <typename T, int B, bool DEFL>
__global__ __launch_bounds__(kThreads) void k_true_residual(PcgArgs<T> a, int init, int has_x0) {
    __shared__ double sm[4 * kMaxRhs];
    int32_t sys;
    int64_t r0, r1;
    block_rows(a.gs, a.rpb, a.N, sys, r0, r1);
    const int k = threadIdx.x % B;
    const int sidx = sys * B + k;
    const bool on = (a.mask >> sidx) & 1u;
    const double* __restrict__ vals = a.vals64 + (int64_t)sys * a.s.len;
    const T* __restrict__ dinv = a.dinv + (int64_t)sys * a.N;
    const double* __restrict__ b = a.b64 + (int64_t)sys * a.N * B;
    const double* __restrict__ x64 = a.x64 + (int64_t)sys * a.N * B;
    T* __restrict__ r = a.r + (int64_t)sys * a.N * B;
    T* __restrict__ pa = a.pa + (int64_t)sys * a.N * B;
    T* __restrict__ xl = a.x + (int64_t)sys * a.N * B;
    const int32_t* __restrict__ cols = a.s.cols;
    double rr = 0.0, rz = 0.0, z1 = 0.0, r1s = 0.0, bb = 0.0;
    if (on) {
        for (int64_t row = r0 + threadIdx.x / B; row < r1; row += kThreads / B) {
            const int64_t idx = row * B + k;
            double res = b[idx];
            if (init) bb += res * res;
            if (!init || has_x0) {
                double sum = 0.0;
                if (a.u64) {
                    // stencil form: U_0 x_i + sum_j U_j[i] x_{i+u_j} + U_j[i-u_j] x_{i-u_j}
                    const int M1 = a.m + 1;
                    const double* __restrict__ U = a.u64 + (int64_t)sys * a.N * M1;
                    const int32_t i = static_cast<int32_t>(row);
                    const int32_t ix = i % a.nx, iy = (i / a.nx) % a.ny, iz = i / (a.nx * a.ny);
                    sum = U[(int64_t)i * M1] * x64[idx];
                    for (int j = 0; j < a.m; ++j) {
                        const int4 t = a.tab[j];
                        const int32_t ux = ix + t.x, uy = iy + t.y, uz = iz + t.z;
                        if (ux >= 0 && ux < a.nx && uy >= 0 && uy < a.ny && uz < a.nz)
                            sum += U[(int64_t)i * M1 + j + 1] * x64[(int64_t)(i + t.w) * B + k];
                        const int32_t lx = ix - t.x, ly = iy - t.y, lz = iz - t.z;
                        if (lx >= 0 && lx < a.nx && ly >= 0 && ly < a.ny && lz >= 0)
                            sum += U[(int64_t)(i - t.w) * M1 + j + 1] * x64[(int64_t)(i - t.w) * B + k];
                    }
                } else {
                    const int32_t base = a.s.slice_ptr[row / kSlice] + static_cast<int32_t>(row % kSlice);
                    const int32_t n = a.s.rowlen[row];
                    for (int32_t j = 0; j < n; ++j) {
                        const int32_t col = cols[base + j * kSlice];
                        sum += vals[base + j * kSlice] * x64[(int64_t)col * B + k];
                    }
                }
                res -= sum;
            }
            const T rl = static_cast<T>(res);
            r[idx] = rl;
            if (init) {
                pa[idx] = T(0);
                if ((void*)xl != (void*)x64) xl[idx] = T(0);
            }
            const T zi = dinv[row] * rl;
            rr += res * res;
            rz += static_cast<double>(rl) * static_cast<double>(zi);
            if (DEFL) {
                z1 += static_cast<double>(zi);
                r1s += static_cast<double>(rl);
            }
        }
    }
    const int S = a.nsys * B;
    double v0 = block_sum<B>(rr, sm);
    double v1 = block_sum<B>(rz, sm);
    double v2 = block_sum<B>(z1, sm);
    double v3 = block_sum<B>(r1s, sm);
    double v4 = block_sum<B>(bb, sm);
    if (threadIdx.x < B) {
        const int v = sys * B + threadIdx.x;
        write_partial(a.partials, v, a.gs, v0);
        write_partial(a.partials, S + v, a.gs, v1);
        write_partial(a.partials, 2 * S + v, a.gs, v2);
        write_partial(a.partials, 3 * S + v, a.gs, v3);
        write_partial(a.partials, 4 * S + v, a.gs, v4);
    }
}

// ---------------------------------------------------------------- reductions
// One block of kRedThreads threads sums the per-block partials of the kernel
// that ran before it, in a fixed order, and updates the scalars. Kernel
// boundaries order everything: no atomics, no inter-block waiting.
constexpr int kRedThreads = 1024;

struct RedArgs {
    PcgScal* sc;
    PcgShared* sh;
    const double* partials;
    int32_t gs;
    int32_t S;
    int64_t N;
    double rtol2;
    int32_t maxit;
    uint32_t mask;
    int32_t init;
};

// out[v] = sum_b partials[v * gs + b] for v < nv, in shared memory
__device__ void reduce_rows(const double* partials, int nv, int gs, double* out) {
    int tpv = 64;
    while (tpv * nv > kRedThreads && tpv > 1) tpv >>= 1;
    const int vpp = kRedThreads / tpv;
    for (int v0 = 0; v0 < nv; v0 += vpp) {
        const int v = v0 + threadIdx.x / tpv;
        const int sub = threadIdx.x % tpv;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        if (v < nv) {
            const double* P = partials + (int64_t)v * gs;
            int b = sub;
            for (; b + 3 * tpv < gs; b += 4 * tpv) {
                s0 += P[b];
                s1 += P[b + tpv];
                s2 += P[b + 2 * tpv];
                s3 += P[b + 3 * tpv];
            }
            for (; b < gs; b += tpv) s0 += P[b];
        }
        double sum = (s0 + s1) + (s2 + s3);
        for (int off = tpv >> 1; off >= 1; off >>= 1) sum += __shfl_xor(sum, off);
        if (sub == 0 && v < nv) out[v] = sum;
    }
    __syncthreads();
}

// after direction+SpMV: alpha = r.z / p.q; the new p becomes current
__global__ __launch_bounds__(kRedThreads) void k_red_alpha(RedArgs a) {
    __shared__ double tot[kMaxSys];
    if (a.sh->n_active == 0) return;
    reduce_rows(a.partials, a.S, a.gs, tot);
    if (threadIdx.x < a.S) {
        PcgScal& c = a.sc[threadIdx.x];
        if (c.active) {
            c.pq = tot[threadIdx.x];
            c.alpha = c.pq != 0.0 ? c.rz / c.pq : 0.0;
        } else {
            c.alpha = 0.0;
        }
    }
    if (threadIdx.x == 0) a.sh->parity ^= 1;
}

// after the update: beta, convergence flags, iteration counts
template <bool DEFL>
__global__ __launch_bounds__(kRedThreads) void k_red_beta(RedArgs a) {
    __shared__ double tot[4 * kMaxSys];
    if (a.sh->n_active == 0) return;
    constexpr int Q = DEFL ? 4 : 2;
    const int S = a.S;
    reduce_rows(a.partials, Q * S, a.gs, tot);
    if (threadIdx.x < S) {
        PcgScal& c = a.sc[threadIdx.x];
        if (c.active) {
            double rzn = tot[threadIdx.x];
            const double rrn = tot[S + threadIdx.x];
            double cn = 0.0;
            if (DEFL) {
                cn = tot[2 * S + threadIdx.x] / static_cast<double>(a.N);
                rzn -= cn * tot[3 * S + threadIdx.x];
            }
            c.beta = c.rz != 0.0 ? rzn / c.rz : 0.0;
            c.rz_prev = c.rz;
            c.rz = rzn;
            c.c = cn;
            c.rr = rrn;
            c.iters += 1;
            if (rrn <= a.rtol2 * c.bnorm2 || !(rrn == rrn)) {
                c.active = 0;
                c.pending = 1;
            } else if (c.iters >= a.maxit) {
                c.active = 0;
            }
        }
    }
    __syncthreads();
    count_active(a.sc, a.sh, S);
}
// after a true-residual recomputation (or the set-up of a run)
template <bool DEFL>
__global__ __launch_bounds__(kRedThreads) void k_red_true(RedArgs a) {
    __shared__ double tot[5 * kMaxSys];
    const int S = a.S;
    const int init = a.init;
    reduce_rows(a.partials, 5 * S, a.gs, tot);
    if (threadIdx.x < S && ((a.mask >> threadIdx.x) & 1u)) {
        PcgScal& c = a.sc[threadIdx.x];
        const double rrt = tot[threadIdx.x];
        double rzn = tot[S + threadIdx.x];
        double cn = 0.0;
        if (DEFL) {
            cn = tot[2 * S + threadIdx.x] / static_cast<double>(a.N);
            rzn -= cn * tot[3 * S + threadIdx.x];
        }
        if (init) {
            // bnorm2 of the deflated run is set by the mean kernel (norm of the
            // unprojected right-hand side)
            if (!DEFL) c.bnorm2 = tot[4 * S + threadIdx.x];
            c.iters = 0;
            c.updates = 0;
            c.beta = 0.0;
            c.rz_prev = rzn;
            c.rz = rzn;
        } else {
            // the residual replaced here is the recursive one's continuation only
            // while the two agree; one far above it (a failed convergence check,
            // or FP32 drift past a reliable-update point) would scale the old
            // direction by rz_true / rz_prev and stall the iteration, so the lane
            // restarts from the true residual (beta = 0: p = z)
            const bool stale = rrt > 4.0 * c.rr;
            c.beta = (!stale && c.rz_prev != 0.0) ? rzn / c.rz_prev : 0.0;
            c.rz = rzn;
            c.updates += 1;
        }
        c.c = cn;
        c.rr = rrt;
        c.truerr = rrt;
        c.rlast2 = rrt;
        c.pending = 0;
        if (rrt <= a.rtol2 * c.bnorm2) {
            c.done = 1;
            c.active = 0;
        } else if (c.iters >= a.maxit) {
            c.done = 0;
            c.active = 0;
        } else {
            c.done = 0;
            c.active = 1;
        }
    }
    __syncthreads();
    count_active(a.sc, a.sh, S);
    if (threadIdx.x == 0) {
        if (init) a.sh->parity = 0;
    }
}
// deflation: mean of each block of b, b <- b - mean, sc.mean = mean / delta,
// sc.bnorm2 = ||b||^2 before projection (B = 1). Three kernels: per-block
// partial sums, one block finishing them in order, the subtraction.
constexpr int kDeflBlocks = 256;

__global__ __launch_bounds__(kThreads) void k_defl_partials(const double* __restrict__ b64, int64_t N,
                                                            double* __restrict__ part) {
    __shared__ double sm[4];
    const int sys = blockIdx.y;
    const double* b = b64 + (int64_t)sys * N;
    const int64_t chunk = (N + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk;
    const int64_t i1 = i0 + chunk < N ? i0 + chunk : N;
    double s = 0.0, s2 = 0.0;
    for (int64_t i = i0 + threadIdx.x; i < i1; i += kThreads) {
        s += b[i];
        s2 += b[i] * b[i];
    }
    s = block_sum<1>(s, sm);
    s2 = block_sum<1>(s2, sm);
    if (threadIdx.x == 0) {
        part[(sys * 2) * gridDim.x + blockIdx.x] = s;
        part[(sys * 2 + 1) * gridDim.x + blockIdx.x] = s2;
    }
}

__global__ void k_defl_finish(const double* __restrict__ part, int nb, int64_t N, int nsys, PcgScal* sc,
                              double inv_delta) {
    if (threadIdx.x != 0) return;
    for (int sys = 0; sys < nsys; ++sys) {
        double s = 0.0, s2 = 0.0;
        for (int b = 0; b < nb; ++b) {
            s += part[(sys * 2) * nb + b];
            s2 += part[(sys * 2 + 1) * nb + b];
        }
        const double mean = s / static_cast<double>(N);
        sc[sys].mean = mean * inv_delta;
        sc[sys].c = mean;          // temporarily: the mean to subtract
        sc[sys].bnorm2 = s2;
        sc[sys].done = 0;
        sc[sys].active = 0;
        sc[sys].pending = 0;
    }
}

__global__ void k_defl_subtract(double* __restrict__ b64, int64_t N, const PcgScal* __restrict__ sc) {
    const int sys = blockIdx.y;
    const double m = sc[sys].c;
    double* b = b64 + (int64_t)sys * N;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        b[i] -= m;
}

__global__ void k_deactivate(PcgScal* sc, int S, PcgShared* sh, uint32_t mask) {
    if (threadIdx.x != 0) return;
    int n = 0;
    for (int i = 0; i < S; ++i) {
        if ((mask >> i) & 1u) sc[i].active = 0;
        n += sc[i].active;
    }
    sh->n_active = n;
}

__global__ void k_reset_scal(PcgScal* sc, int S, PcgShared* sh) {
    int i = threadIdx.x;
    if (i < S) {
        sc[i].done = 0;
        sc[i].active = 0;
        sc[i].pending = 0;
        sc[i].iters = 0;
        sc[i].updates = 0;
        sc[i].mean = 0.0;
        sc[i].alpha = 0.0;
    }
    if (i == 0) {
        sh->counter = 0u;
        sh->parity = 0;
        sh->n_active = 0;
    }
}

// y = A64 x + shift x for nsys systems, B right-hand sides
template <int B>
__global__ __launch_bounds__(kThreads) void k_spmv64(const Sell s, int64_t N, const double* __restrict__ vals,
                                                    const double* __restrict__ x, double* __restrict__ y,
                                                    double shift) {
    const int sys = blockIdx.y;
    const int k = threadIdx.x % B;
    const double* V = vals + (int64_t)sys * s.len;
    const double* X = x + (int64_t)sys * N * B;
    double* Y = y + (int64_t)sys * N * B;
    for (int64_t row = blockIdx.x * (int64_t)(kThreads / B) + threadIdx.x / B; row < N;
         row += (int64_t)gridDim.x * (kThreads / B)) {
        const int32_t base = s.slice_ptr[row / kSlice] + static_cast<int32_t>(row % kSlice);
        const int32_t n = s.rowlen[row];
        double sum = 0.0;
        for (int32_t j = 0; j < n; ++j) sum += V[base + j * kSlice] * X[(int64_t)s.cols[base + j * kSlice] * B + k];
        Y[row * B + k] = sum + shift * X[row * B + k];
    }
}

// ---------------------------------------------------------------- host side
// number of launched iterations of a chunk that did work: the largest
// per-lane iteration increase
inline int live_iters(const PcgScal* hs, int S, const std::vector<int>& before, int chunk) {
    int m = 0;
    for (int i = 0; i < S; ++i) m = std::max(m, hs[i].iters - before[i]);
    return std::min(m, chunk);
}

template <typename T>
RedArgs red_args(const PcgArgs<T>& a, int S, uint32_t mask = 0, int init = 0) {
    RedArgs r{};
    r.sc = a.sc;
    r.sh = a.sh;
    r.partials = a.partials;
    r.gs = a.gs;
    r.S = S;
    r.N = a.N;
    r.rtol2 = a.rtol2;
    r.maxit = a.maxit;
    r.mask = mask;
    r.init = init;
    return r;
}

// Per-thread register budgets of the stencil kernel: NPF halo-plane elements
// (and output elements) per thread, NPU staged diagonal values per thread
// (0: diagonals read from global memory), TX0 the preferred tile width.
template <typename T, int B>
struct StTile {
    static constexpr int NPF = B == 16 ? (sizeof(T) == 4 ? 6 : 4) : (B >= 4 ? 4 : (B == 2 ? 2 : 1));
    static constexpr int NU = B == 16 ? (sizeof(T) == 4 ? 3 : 2) : (B == 8 ? 4 : 8);
    static constexpr int HX = B >= 16 ? 17 : (B == 8 ? 18 : 34);   // halo'd tile width of the Kuhn kernel
    static constexpr size_t LDS = (size_t)3 * (NPF + NU) * kStThreads * sizeof(T);
};

template <typename T, int B, bool DEFL, bool KUHN>
const void* stencil_kernel() {
    using TL = StTile<T, B>;
    return reinterpret_cast<const void*>(&k_dir_stencil<T, B, DEFL, TL::NPF, TL::NU, KUHN ? TL::HX : 0>);
}

// one PCG iteration: direction+SpMV, alpha, update, beta
template <typename T, int B, bool DEFL>
inline void launch_iteration(const PcgArgs<T>& a, const StArgs<T>& g, dim3 grid, dim3 blk, hipStream_t st,
                             hipEvent_t* ev) {
    const RedArgs ra = red_args(a, a.nsys * B);
    if (ev) (void)hipEventRecord(ev[0], st);
    using TL = StTile<T, B>;
    if (g.on && g.kuhn)
        hipLaunchKernelGGL((k_dir_stencil<T, B, DEFL, TL::NPF, TL::NU, TL::HX>), grid, dim3(kStThreads), TL::LDS, st,
                           a, g);
    else if (g.on)
        hipLaunchKernelGGL((k_dir_stencil<T, B, DEFL, TL::NPF, TL::NU, 0>), grid, dim3(kStThreads), TL::LDS, st, a,
                           g);
    else
        hipLaunchKernelGGL((k_dir_spmv<T, B, DEFL>), grid, blk, 0, st, a);
    if (ev) (void)hipEventRecord(ev[1], st);
    hipLaunchKernelGGL(k_red_alpha, dim3(1), dim3(kRedThreads), 0, st, ra);
    if (ev) (void)hipEventRecord(ev[2], st);
    if (g.on)
        hipLaunchKernelGGL((k_update<T, B, DEFL, true>), grid, blk, 0, st, a);
    else
        hipLaunchKernelGGL((k_update<T, B, DEFL, false>), grid, blk, 0, st, a);
    if (ev) (void)hipEventRecord(ev[3], st);
    hipLaunchKernelGGL(k_red_beta<DEFL>, dim3(1), dim3(kRedThreads), 0, st, ra);
    if (ev) (void)hipEventRecord(ev[4], st);
}

template <typename T, int B, bool DEFL>
inline void launch_true_residual(const PcgArgs<T>& a, dim3 grid, dim3 blk, hipStream_t st, int init, int has_x0) {
    hipLaunchKernelGGL((k_true_residual<T, B, DEFL>), grid, blk, 0, st, a, init, has_x0);
    hipLaunchKernelGGL(k_red_true<DEFL>, dim3(1), dim3(kRedThreads), 0, st, red_args(a, a.nsys * B, a.mask, init));
}

// Captured graph of `chunk` PCG iterations for this kernel configuration. The
// capture runs on a private stream (capture is not allowed on the legacy
// default stream); replays go to the context's stream.
template <typename T, int B, bool DEFL>
qpat_status chunk_graph(qpat_ctx* c, const PcgArgs<T>& a, const StArgs<T>& g, int chunk, dim3 grid, dim3 blk,
                        hipGraphExec_t* out) {
    const void* kfn = !g.on ? reinterpret_cast<const void*>(&k_dir_spmv<T, B, DEFL>)
                      : g.kuhn ? stencil_kernel<T, B, DEFL, true>() : stencil_kernel<T, B, DEFL, false>();
    char key[256];
    snprintf(key, sizeof key, "%p/%d/%d/%d/%.17g/%d/%d/%p/%d/%d/%d/%d", kfn, chunk, a.gs, a.nsys, a.rtol2, a.maxit,
             (int)a.N, (const void*)g.U, g.hx, g.hy, g.zc, g.items);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return QPAT_OK;
    }
    if (!c->cap_stream) QPAT_HIP(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    QPAT_HIP(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    for (int i = 0; i < chunk; ++i) launch_iteration<T, B, DEFL>(a, g, grid, blk, c->cap_stream, nullptr);
    QPAT_HIP(c, hipStreamEndCapture(c->cap_stream, &graph));
    hipGraphExec_t exec = nullptr;
    QPAT_HIP(c, hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    QPAT_HIP(c, hipGraphDestroy(graph));
    c->graphs[key] = exec;
    *out = exec;
    return QPAT_OK;
}

// Tiling of the stencil kernel for this launch (g->on = false keeps the
// sliced-ELL kernel): the largest tile that fits the register and LDS
// budgets, then the number of z chunks that best balances the work items
// over the blocks resident per XCD.
template <typename T, int B, bool DEFL>
qpat_status make_st(qpat_ctx* c, Op op, const PcgArgs<T>& a, StArgs<T>* out) {
    StArgs<T> g{};
    g.on = false;
    *out = g;
    const Lattice& L = c->lat;
    if (!L.on || c->opts.operator_format != 1) return QPAT_OK;
    using TL = StTile<T, B>;
    const int64_t sz = sizeof(T);
    // 32-bit byte offsets below kOut: every array the kernel addresses under 2 GiB
    if ((int64_t)(L.m + 1) * c->N * sz >= (int64_t(1) << 31) || c->N * B * sz >= (int64_t(1) << 31)) return QPAT_OK;
    bool kuhn = L.m == kKuhnM;
    for (int j = 0; kuhn && j < kKuhnM; ++j)
        kuhn = L.dx[j] == kKdx[j] && L.dy[j] == kKdy[j] && L.dz[j] == kKdz[j];
    const int64_t hn_max = std::min<int64_t>((int64_t)TL::NPF * kStThreads / B,
                                             (int64_t)TL::NU * kStThreads / (L.m + 1));
    int64_t hx = TL::HX;
    if (!kuhn) {
        const int64_t tiles_x = (L.nx + TL::HX - 3) / (TL::HX - 2);
        hx = (L.nx + tiles_x - 1) / tiles_x + 2;
    }
    if (hx > hn_max / 3) {
        if (kuhn) kuhn = false;
        hx = hn_max / 3;
    }
    if (hx < 3) return QPAT_OK;
    int64_t ty = std::min<int64_t>(hn_max / hx - 2, L.ny);
    if (ty < 1) return QPAT_OK;
    const int64_t tiles_y = (L.ny + ty - 1) / ty;
    ty = (L.ny + tiles_y - 1) / tiles_y;
    const int64_t tiles_x = (L.nx + hx - 3) / (hx - 2);
    g.kuhn = kuhn;
    g.nx = L.nx;
    g.ny = L.ny;
    g.nz = L.nz;
    g.m = L.m;
    g.tab = reinterpret_cast<const int4*>(c->lat_tab);
    g.hx = static_cast<int32_t>(hx);
    g.hy = static_cast<int32_t>(ty + 2);
    g.tiles_x = static_cast<int32_t>(tiles_x);
    g.tiles_y = static_cast<int32_t>(tiles_y);
    static_assert(TL::LDS <= 159 * 1024, "stencil LDS budget");
    const void* kfn = kuhn ? stencil_kernel<T, B, DEFL, true>() : stencil_kernel<T, B, DEFL, false>();
    char key[96];
    snprintf(key, sizeof key, "st/%p", kfn);
    int occ = 0;
    auto it = c->st_occ.find(key);
    if (it != c->st_occ.end()) {
        occ = it->second;
    } else {
        // dynamic LDS beyond the default per-block limit has to be allowed per kernel
        QPAT_HIP(c, hipFuncSetAttribute(kfn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)TL::LDS));
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kfn, kStThreads, TL::LDS) != hipSuccess) occ = 1;
        c->st_occ[key] = occ;
    }
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) cus = 256;
    const int64_t slots = (int64_t)std::max(occ, 1) * std::max(cus / 8, 1);
    const int64_t conc = std::min<int64_t>(slots, (int64_t)(a.gs / 8) * a.nsys);
    const int64_t tiles = tiles_x * tiles_y;
    int64_t best = -1, best_zc = L.nz;
    for (int64_t nch = 1; nch <= L.nz; ++nch) {
        const int64_t zc = (L.nz + nch - 1) / nch;
        const int64_t items = tiles * ((L.nz + zc - 1) / zc);
        const int64_t wx = (items + 7) / 8;
        const int64_t cost = ((wx * a.nsys + conc - 1) / conc) * (zc + 2);
        if (best < 0 || cost < best) {
            best = cost;
            best_zc = zc;
        }
    }
    g.zc = static_cast<int32_t>(best_zc);
    g.items = static_cast<int32_t>(tiles * ((L.nz + best_zc - 1) / best_zc));
    const bool is64 = std::is_same<T, double>::value;
    if (op == Op::K)
        g.U = is64 ? reinterpret_cast<const T*>(c->KU64) : reinterpret_cast<const T*>(c->KU32);
    else if (is64)
        g.U = reinterpret_cast<const T*>(c->MU64);
    else
        return QPAT_OK;
    g.on = true;
    *out = g;
    return QPAT_OK;
}

template <typename T, int B, bool DEFL>
struct Runner {
    static qpat_status run(qpat_ctx* c, Op op, PcgArgs<T>& a, double rtol, SolveStats* st, bool has_x0) {
        const int S = a.nsys * B;
        const dim3 grid(a.gs * a.nsys), blk(kThreads);
        StArgs<T> g{};
        QPAT_TRY((make_st<T, B, DEFL>(c, op, a, &g)));
        hipStream_t sm = c->stream;
        hipLaunchKernelGGL(k_reset_scal, dim3(1), dim3(64), 0, sm, a.sc, S, a.sh);
        if (DEFL) {
            hipLaunchKernelGGL(k_defl_partials, dim3(kDeflBlocks, a.nsys), blk, 0, sm, a.b64, a.N, a.partials);
            hipLaunchKernelGGL(k_defl_finish, dim3(1), dim3(64), 0, sm, a.partials, kDeflBlocks, a.N, a.nsys, a.sc,
                               a.inv_delta);
            hipLaunchKernelGGL(k_defl_subtract, dim3(grid_for(a.N, kThreads, 4096), a.nsys), blk, 0, sm, a.b64, a.N,
                               a.sc);
        }
        if (!has_x0) QPAT_HIP(c, hipMemsetAsync(a.x64, 0, sizeof(double) * a.N * B * a.nsys, sm));
        a.mask = (S >= 32) ? 0xffffffffu : ((1u << S) - 1u);
        launch_true_residual<T, B, DEFL>(a, grid, blk, sm, 1, has_x0 ? 1 : 0);
        QPAT_HIP(c, hipGetLastError());
        PcgScal* hs = c->scal_host;
        // the stencil direction kernel applies x += alpha p one iteration late;
        // apply what is pending before x is read (fold, true residual, result)
        auto flush = [&]() {
            hipLaunchKernelGGL((k_xflush<T, B>), grid, blk, 0, sm, a);
            hipLaunchKernelGGL(k_alpha_done, dim3(1), dim3(64), 0, sm, a.sc, S);
        };
        auto fetch = [&]() -> qpat_status {
            QPAT_HIP(c, hipMemcpyAsync(hs, a.sc, sizeof(PcgScal) * S, hipMemcpyDeviceToHost, sm));
            QPAT_HIP(c, hipStreamSynchronize(sm));
            return QPAT_OK;
        };
        QPAT_TRY(fetch());
        const bool mixed = !std::is_same<T, double>::value;
        const double ru2 = c->opts.ru_delta * c->opts.ru_delta;
        int chunk = 16;
        std::vector<double> best_true(S, INFINITY);
        std::vector<int> stalls(S, 0);
        std::vector<double> rr_prev(S);
        for (int i = 0; i < S; ++i) rr_prev[i] = hs[i].rr;
        std::vector<int> iters_before(S);
        for (;;) {
            for (int i = 0; i < S; ++i) iters_before[i] = hs[i].iters;
            bool any_active = false;
            for (int i = 0; i < S; ++i) any_active |= hs[i].active != 0;
            if (!any_active) break;
            const bool prof = c->prof_on;
            if (prof && c->ev_pool.size() < (size_t)5 * chunk) {
                size_t old = c->ev_pool.size();
                c->ev_pool.resize((size_t)5 * chunk);
                for (size_t e = old; e < c->ev_pool.size(); ++e) QPAT_HIP(c, hipEventCreate(&c->ev_pool[e]));
            }
            if (!prof && c->opts.use_graphs) {
                // replay a captured graph of `chunk` iterations (kernel arguments are
                // identical from one iteration to the next: all state is on the device)
                hipGraphExec_t gx = nullptr;
                QPAT_TRY((chunk_graph<T, B, DEFL>(c, a, g, chunk, grid, blk, &gx)));
                QPAT_HIP(c, hipGraphLaunch(gx, sm));
            } else {
                for (int it = 0; it < chunk; ++it)
                    launch_iteration<T, B, DEFL>(a, g, grid, blk, sm, prof ? &c->ev_pool[5 * it] : nullptr);
            }
            QPAT_HIP(c, hipGetLastError());
            QPAT_TRY(fetch());
            if (prof) {
                // launches after every lane stopped exit at once; count only live ones
                const int base = op == Op::K ? 0 : 2;
                for (int it = 0; it < chunk; ++it) {
                    float t1 = 0.f, t2 = 0.f;
                    QPAT_HIP(c, hipEventElapsedTime(&t1, c->ev_pool[5 * it], c->ev_pool[5 * it + 1]));
                    QPAT_HIP(c, hipEventElapsedTime(&t2, c->ev_pool[5 * it + 2], c->ev_pool[5 * it + 3]));
                    if (it >= live_iters(hs, S, iters_before, chunk)) break;
                    int lanes = 0;
                    for (int i = 0; i < S; ++i) lanes += (hs[i].iters - iters_before[i]) > it;
                    for (int kk = 0; kk < 2; ++kk) {
                        qpat_kstat& ks = c->prof[base + kk];
                        const double t = kk == 0 ? t1 : t2;
                        ks.launches += 1;
                        ks.lanes += lanes;
                        ks.total_ms += t;
                        ks.min_ms = ks.launches == 1 ? t : std::min(ks.min_ms, t);
                        ks.max_ms = std::max(ks.max_ms, t);
                    }
                }
            }
            uint32_t mask = 0;
            for (int i = 0; i < S; ++i) {
                if (hs[i].pending) mask |= 1u << i;
                else if (mixed && hs[i].active && hs[i].rr <= ru2 * hs[i].rlast2) mask |= 1u << i;
            }
            if (mask && mixed) {
                // a recomputation is due anyway: take along the lanes within 10x (in
                // norm) of their own reliable-update point, so the block's lanes stay
                // in step and share later recomputations (each costs a full FP64 SpMV)
                for (int i = 0; i < S; ++i)
                    if (hs[i].active && !hs[i].pending && hs[i].rr <= 100.0 * ru2 * hs[i].rlast2) mask |= 1u << i;
            }
            if (mask) {
                const uint32_t confirm = mask & [&] {
                    uint32_t m = 0;
                    for (int i = 0; i < S; ++i)
                        if (hs[i].pending) m |= 1u << i;
                    return m;
                }();
                a.mask = mask;
                if (g.on) flush();
                if (mixed) hipLaunchKernelGGL((k_fold<T, B>), grid, blk, 0, sm, a);
                launch_true_residual<T, B, DEFL>(a, grid, blk, sm, 0, 0);
                QPAT_HIP(c, hipGetLastError());
                QPAT_TRY(fetch());
                // a confirmation that failed without halving the best true residual
                // counts as a stall; three stalls end the lane (QPAT_ERR_NOCONV)
                uint32_t stop = 0;
                for (int i = 0; i < S; ++i) {
                    if (!((confirm >> i) & 1u) || hs[i].done) continue;
                    if (hs[i].truerr < 0.25 * best_true[i]) {
                        best_true[i] = hs[i].truerr;
                        stalls[i] = 0;
                    } else if (++stalls[i] >= 3) {
                        stop |= 1u << i;
                    }
                }
                if (stop) {
                    hipLaunchKernelGGL(k_deactivate, dim3(1), dim3(64), 0, sm, a.sc, S, a.sh, stop);
                    QPAT_TRY(fetch());
                }
            }
            // next chunk: predicted iterations to the nearest target of the slowest lane
            int need = 4;
            for (int i = 0; i < S; ++i) {
                if (!hs[i].active) continue;
                double target = rtol * rtol * hs[i].bnorm2;
                if (mixed) target = std::max(target, ru2 * hs[i].rlast2);
                double rate = (rr_prev[i] > 0 && hs[i].rr > 0 && hs[i].rr < rr_prev[i])
                                  ? std::log(hs[i].rr / rr_prev[i]) / chunk : 0.0;
                int pred = rate < 0 ? static_cast<int>(std::log(target / hs[i].rr) / rate) + 1 : 64;
                need = std::max(need, pred);
            }
            // mixed precision: the FP32 recursive residual may not run far past a
            // reliable-update point (its drift grows with the distance), and CG
            // often speeds up, so chunks stay short there
            chunk = std::min(std::max(need, 4), mixed ? 32 : 256);
            if (c->opts.use_graphs) {
                int p2 = 4;
                while (p2 < chunk) p2 <<= 1;
                chunk = p2;
            }
            for (int i = 0; i < S; ++i) rr_prev[i] = hs[i].rr;
        }
        if (g.on) flush();
        if (mixed) {
            // fold anything left (lanes stopped at maxit)
            uint32_t mask = 0;
            for (int i = 0; i < S; ++i)
                if (!hs[i].done) mask |= 1u << i;
            if (mask) {
                a.mask = mask;
                hipLaunchKernelGGL((k_fold<T, B>), grid, blk, 0, sm, a);
            }
        }
        for (int i = 0; i < S; ++i) {
            const double rel = hs[i].bnorm2 > 0 ? std::sqrt(hs[i].truerr / hs[i].bnorm2) : 0.0;
            st->add(hs[i].iters, rel, hs[i].updates, hs[i].done != 0);
        }
        return QPAT_OK;
    }
};

template <typename T, bool DEFL>
qpat_status dispatch_B(qpat_ctx* c, Op op, int B, PcgArgs<T>& a, double rtol, SolveStats* st, bool x0) {
    switch (B) {
        case 1: return Runner<T, 1, DEFL>::run(c, op, a, rtol, st, x0);
        case 2: return Runner<T, 2, DEFL>::run(c, op, a, rtol, st, x0);
        case 4: return Runner<T, 4, DEFL>::run(c, op, a, rtol, st, x0);
        case 8: return Runner<T, 8, DEFL>::run(c, op, a, rtol, st, x0);
        case 16: return Runner<T, 16, DEFL>::run(c, op, a, rtol, st, x0);
        default: return fail(c, QPAT_ERR_ARG, "block size %d not supported", B);
    }
}

template <typename T, int B, bool DEFL>
int occupancy_of() {
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void*>(&k_dir_spmv<T, B, DEFL>),
                                                     kThreads, 0) != hipSuccess)
        blocks = 4;
    return blocks;
}

// resident blocks of the direction+SpMV kernel over the whole device (cached)
int resident_blocks(qpat_ctx* c, bool defl, bool fp64, int B) {
    const int key = (defl ? 100 : 0) + (fp64 ? 50 : 0) + B;
    auto it = c->occupancy.find(key);
    if (it != c->occupancy.end()) return it->second;
    int cus = 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) cus = 256;
    int per_cu = 4;
    if (defl) per_cu = occupancy_of<double, 1, true>();
    else if (fp64) {
        switch (B) {
            case 1: per_cu = occupancy_of<double, 1, false>(); break;
            case 2: per_cu = occupancy_of<double, 2, false>(); break;
            case 4: per_cu = occupancy_of<double, 4, false>(); break;
            case 8: per_cu = occupancy_of<double, 8, false>(); break;
            default: per_cu = occupancy_of<double, 16, false>(); break;
        }
    } else {
        switch (B) {
            case 1: per_cu = occupancy_of<float, 1, false>(); break;
            case 2: per_cu = occupancy_of<float, 2, false>(); break;
            case 4: per_cu = occupancy_of<float, 4, false>(); break;
            case 8: per_cu = occupancy_of<float, 8, false>(); break;
            default: per_cu = occupancy_of<float, 16, false>(); break;
        }
    }
    const int r = std::max(per_cu, 1) * cus;
    c->occupancy[key] = r;
    return r;
}

template <typename T>
PcgArgs<T> make_args(qpat_ctx* c, Op op, int B) {
    PcgArgs<T> a{};
    a.s = c->sell;
    a.N = c->N;
    a.nsys = op == Op::Prior ? 2 : 1;
    // one resident wave of blocks: occupancy of the direction+SpMV kernel times
    // the compute units, split over the systems, a multiple of 8 (XCD mapping)
    const int64_t rows_per_pass = kThreads / B;
    int64_t want = (c->N + rows_per_pass - 1) / rows_per_pass;
    int64_t cap = resident_blocks(c, op == Op::Prior, std::is_same<T, double>::value, B) / a.nsys;
    int64_t gs = std::min(want, std::max<int64_t>(cap, 8));
    gs = ((gs + 7) / 8) * 8;
    gs = std::min<int64_t>(gs, kMaxBlocks);   // size of the partial-sum buffer
    int64_t rpb = (c->N + gs - 1) / gs;
    rpb = ((rpb + kSlice - 1) / kSlice) * kSlice;
    a.gs = static_cast<int32_t>(gs);
    a.rpb = static_cast<int32_t>(rpb);
    const bool is64 = std::is_same<T, double>::value;
    if (op == Op::K) {
        a.vals = is64 ? reinterpret_cast<const T*>(c->K64) : reinterpret_cast<const T*>(c->K32);
        a.dinv = is64 ? reinterpret_cast<const T*>(c->Kdinv64) : reinterpret_cast<const T*>(c->Kdinv32);
        a.vals64 = c->K64;
        a.dinv64 = c->Kdinv64;
        a.u64 = c->KU64;
    } else {
        a.vals = is64 ? reinterpret_cast<const T*>(c->M64) : reinterpret_cast<const T*>(c->M32);
        a.dinv = is64 ? reinterpret_cast<const T*>(c->Mdinv64) : reinterpret_cast<const T*>(c->Mdinv32);
        a.vals64 = c->M64;
        a.dinv64 = c->Mdinv64;
        a.u64 = c->MU64;
    }
    a.r = static_cast<T*>(c->rl);
    a.pa = static_cast<T*>(c->pa);
    a.pb = static_cast<T*>(c->pb);
    a.q = static_cast<T*>(c->ql);
    a.x = is64 ? reinterpret_cast<T*>(c->x64) : static_cast<T*>(c->xl);
    a.x64 = c->x64;
    a.b64 = c->b64;
    a.sc = c->scal;
    a.sh = c->shared;
    a.partials = c->partials;
    a.inv_delta = c->delta > 0 ? 1.0 / c->delta : 0.0;
    if (c->lat.on && c->opts.operator_format == 1) {
        a.tab = reinterpret_cast<const int4*>(c->lat_tab);
        a.nx = c->lat.nx;
        a.ny = c->lat.ny;
        a.nz = c->lat.nz;
        a.m = c->lat.m;
    } else {
        a.u64 = nullptr;
    }
    return a;
}

}  // namespace

qpat_status pcg_solve(qpat_ctx* c, Op op, int B, SolveStats* st, bool has_x0) {
    const bool mixed = c->opts.precision == 1 && op == Op::K;
    const bool defl = op == Op::Prior && c->opts.prior_deflate;
    const double rtol = op == Op::K ? c->opts.pcg_rtol : c->opts.prior_rtol;
    if (op == Op::Prior) B = 1;
    if (mixed) {
        PcgArgs<float> a = make_args<float>(c, op, B);
        a.rtol2 = rtol * rtol;
        a.maxit = c->opts.pcg_maxit;
        return dispatch_B<float, false>(c, op, B, a, rtol, st, has_x0);
    }
    PcgArgs<double> a = make_args<double>(c, op, B);
    a.rtol2 = rtol * rtol;
    a.maxit = c->opts.pcg_maxit;
    if (defl) return Runner<double, 1, true>::run(c, op, a, rtol, st, false);
    return dispatch_B<double, false>(c, op, B, a, rtol, st, has_x0);
}

qpat_status spmv64(qpat_ctx* c, Op op, int B, const double* x, double* y, double shift) {
    const int nsys = op == Op::Prior ? 2 : 1;
    const double* vals = op == Op::K ? c->K64 : c->M64;
    const dim3 grid(grid_for(c->N, kThreads / B, 4096), nsys), blk(kThreads);
    switch (B) {
        case 1: hipLaunchKernelGGL(k_spmv64<1>, grid, blk, 0, c->stream, c->sell, c->N, vals, x, y, shift); break;
        case 2: hipLaunchKernelGGL(k_spmv64<2>, grid, blk, 0, c->stream, c->sell, c->N, vals, x, y, shift); break;
        case 4: hipLaunchKernelGGL(k_spmv64<4>, grid, blk, 0, c->stream, c->sell, c->N, vals, x, y, shift); break;
        case 8: hipLaunchKernelGGL(k_spmv64<8>, grid, blk, 0, c->stream, c->sell, c->N, vals, x, y, shift); break;
        case 16: hipLaunchKernelGGL(k_spmv64<16>, grid, blk, 0, c->stream, c->sell, c->N, vals, x, y, shift); break;
        default: return fail(c, QPAT_ERR_ARG, "block size %d not supported", B);
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

}  // namespace qpat
