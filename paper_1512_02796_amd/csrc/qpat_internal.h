// Internal definitions of libqpat (HIP, gfx950). Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <algorithm>
#include <cstdio>
#include <map>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/qpat.h"

namespace qpat {

constexpr int kThreads = 256;        // threads per block of every streaming kernel
constexpr int kSlice = 64;           // rows per sliced-ELL slice (one wavefront)
constexpr int kMaxRow = 64;          // longest admissible matrix row
constexpr int kMaxRhs = 16;          // right-hand sides per block solve
constexpr int kMaxSys = 32;          // systems x right-hand sides tracked by one PCG run
constexpr int kTetGeo = 12;          // doubles per tetrahedron: |T|, grad l1, grad l2, grad l3, pad

// Raw buffer access with 32-bit byte offsets: one vector register per
// address, and offsets at or past the resource's size read 0 / are dropped
// (the hardware range check), which handles halo and tile edges.
constexpr uint32_t kOut = 0x80000000u;   // an offset past every resource used here

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), static_cast<short>(0), static_cast<int>(bytes),
                                             0x00020000);
}
template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t b, uint32_t off) {
    if constexpr (sizeof(T) == 4)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(b, off, 0, 0));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(b, off, 0, 0));
}
// the same with the non-temporal hint (cache policy NT): data touched once per pass
__device__ __forceinline__ double bload_nt(__amdgpu_buffer_rsrc_t b, uint32_t off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(b, off, 0, 2));
}
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t b, uint32_t off, double v) {
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b, off, 0, 2);
}
__device__ __forceinline__ void bstore_nt_f32(__amdgpu_buffer_rsrc_t b, uint32_t off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b, off, 0, 2);
}
template <typename T>
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t b, uint32_t off, T v) {
    if constexpr (sizeof(T) == 4)
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), b, off, 0, 0);
    else {
        typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), b, off, 0, 0);
    }
}

struct Error {
    qpat_status st;
    std::string msg;
};

// Sliced ELL of the node-node pattern: slice s covers rows [64 s, 64 s + 64);
// entry k of row i sits at slice_ptr[s] + k * 64 + (i % 64). Padding entries
// have col = i and value 0. Columns are sorted within a row.
struct Sell {
    int64_t N = 0;
    int32_t nslices = 0;
    int64_t len = 0;             // total padded entries
    int32_t max_width = 0;
    int32_t* slice_ptr = nullptr;  // [nslices+1]
    int32_t* slice_w = nullptr;    // [nslices]
    int32_t* rowlen = nullptr;     // [N]
    int32_t* cols = nullptr;       // [len]
    int32_t* diag = nullptr;       // [N] position k of the diagonal in row i
};

// Per (system, right-hand side) scalars of one PCG run; FP64.
struct PcgScal {
    double rz;        // r . z (current)
    double rz_prev;   // r . z before the last update
    double pq;        // p . K p
    double alpha;
    double beta;
    double c;         // deflation: mean of D^{-1} r
    double rr;        // ||r||^2 (recursive)
    double bnorm2;    // ||b||^2
    double rlast2;    // ||r||^2 at the last true-residual recomputation
    double truerr;    // ||b - K x||^2 at the last recomputation
    double mean;      // deflation: mean(b) / delta
    int32_t active;   // 1 while iterating
    int32_t pending;  // 1: recursive residual converged, awaiting a true-residual check
    int32_t done;     // 1: converged on the true residual
    int32_t iters;
    int32_t updates;
    int32_t pad;
};

struct PcgShared {       // device-side counters shared by the kernels of one run
    int32_t n_active;
    int32_t parity;      // which p buffer is current
    uint32_t counter;    // last-block-done counter
    int32_t pad;
};

struct LsqrScal {
    double alpha, beta, rhobar, phibar, rho, phi, theta, c, s;
    double beta1;
    int32_t done;        // lucky breakdown / zero rhs
    int32_t breakdown;   // p.r <= 0 or non-finite
    int32_t steps;
    int32_t rotated;     // 1 when the last step applied a plane rotation
};

// Lattice (stencil) form of the node-node pattern. When node i sits at
// lattice position (i % nx, (i / nx) % ny, i / (nx ny)) and every matrix
// neighbour differs by at most one step along each axis, a symmetric operator
// is stored as its diagonal plus the m "upper" offsets u_1..u_m (dz > 0, or
// dz = 0 and dy > 0, or dz = dy = 0 and dx > 0): U_j[i] = A(i, i + u_j), zero
// where that entry is not in the pattern. Row i then reads
//   A(i, i - u_j) = A(i - u_j, i) = U_j[i - u_j]
// from the partner row. Arrays are [N][m + 1] per system (the m + 1 values of
// a node together), U_0 the diagonal.
constexpr int kMaxUpper = 13;
struct Lattice {
    bool on = false;
    int32_t nx = 0, ny = 0, nz = 0;
    int32_t m = 0;
    int8_t dx[kMaxUpper]{}, dy[kMaxUpper]{}, dz[kMaxUpper]{};
    int8_t code[27]{};     // (dx+1) + 3 (dy+1) + 9 (dz+1) -> 0 diagonal, j >= 1 upper offset j, -1 otherwise
};

struct GuessNet;
struct MgState;

template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
};

}  // namespace qpat

struct qpat_ctx {
    hipStream_t stream = nullptr;
    int device = 0;
    qpat_opts opts{};
    std::string err;

    // mesh
    int64_t N = 0, E = 0, Fb = 0;
    int32_t* tets = nullptr;       // [E][4]
    double* geo = nullptr;         // [E][kTetGeo]
    // geometry classes: when every tetrahedron's geometry equals, bit for bit,
    // one of a few candidates (a uniform lattice with an exactly representable
    // spacing has 6), geo_cls[e] names it and geo_tab holds the candidates
    // ([geo_ncls][kTetGeo]); otherwise geo_cls is null
    uint8_t* geo_cls = nullptr;    // [E]
    double* geo_tab = nullptr;
    int32_t geo_ncls = 0;
    int32_t* bfaces = nullptr;     // [Fb][3]
    double* barea = nullptr;       // [Fb]
    int32_t* n2t_ptr = nullptr;    // [N+1]
    int32_t* n2t = nullptr;        // [4E], entry = e*4 + a
    int32_t* n2f_ptr = nullptr;    // [N+1]
    int32_t* n2f = nullptr;        // [3Fb], entry = f*3 + a
    qpat::Sell sell;
    qpat::Lattice lat;             // stencil form, when the numbering is a lattice
    int32_t* lat_tab = nullptr;    // [kMaxUpper][4]: dx, dy, dz, dx + nx (dy + ny dz)

    // linearisation point and operator
    double* kappa = nullptr;       // [N]
    double* mu = nullptr;          // [N]
    double* K64 = nullptr;         // [sell.len]
    float* K32 = nullptr;
    double* Kdinv64 = nullptr;     // [N]
    float* Kdinv32 = nullptr;
    double* KU64 = nullptr;        // lattice form of K, [N][m+1]
    float* KU32 = nullptr;
    bool have_forward = false;

    // prior
    double* M64 = nullptr;         // [2][sell.len]
    float* M32 = nullptr;
    double* Mdinv64 = nullptr;     // [2][N]  1/(diag + delta)
    float* Mdinv32 = nullptr;
    double* MU64 = nullptr;        // lattice form, [2][N][m+1]
    double delta = 0.0;
    bool have_prior = false;

    // illuminations; data-space vectors are interleaved [N][n_pad]
    int32_t n_ill = 0, n_pad = 0;
    double* f = nullptr;           // [N][n_pad]
    double* phi = nullptr;         // [N][n_pad]

    // PCG workspace, sized for N x kMaxRhs entries per vector
    double* x64 = nullptr;
    double* r64 = nullptr;
    double* b64 = nullptr;
    void* xl = nullptr;            // low-precision iterate (mixed)
    void* rl = nullptr;
    void* pa = nullptr;
    void* pb = nullptr;
    void* ql = nullptr;
    qpat::PcgScal* scal = nullptr; // [kMaxSys]
    qpat::PcgShared* shared = nullptr;
    double* partials = nullptr;    // [4][kMaxSys][max blocks]
    int32_t pcg_blocks = 0;        // blocks per system
    qpat::PcgScal* scal_host = nullptr;  // pinned mirror

    // Jacobian accumulators
    double* acc1 = nullptr;        // [N]
    double* acc2 = nullptr;        // [N]
    double* dvec = nullptr;        // [N][n_pad] scratch in data space
    double* dK = nullptr;          // lattice meshes: dK(s) of J s in the stencil form [N][m+1]
    double* dKc = nullptr;         // [N][2] its coefficients kappa s1, mu s2
    double* tq = nullptr;          // [E] per-tetrahedron sums of J^T t (stiffness part)
    double* tr = nullptr;          // [E][4] per-tetrahedron sums of J^T t (mass part)
    // voxel form of the G kernels (Kuhn lattices of equal voxels): 0 not yet
    // checked against the element form, 1 in use, -1 not applicable
    int32_t vox = -1;
    double vox_h[3] = {0.0, 0.0, 0.0};   // the lattice spacings along x, y, z

    // LSQR
    bool lsqr_ready = false;
    double* lu = nullptr;          // [N][n_pad]
    double* lq = nullptr;          // [N][n_pad]
    double* lw = nullptr;          // W, [N][n_pad]
    double* lv = nullptr;          // [2N]
    double* lwh = nullptr;         // [2N]
    double* lwd = nullptr;         // w direction [2N]
    double* lp = nullptr;          // [2N]
    double* lr = nullptr;          // [2N]
    double* lx = nullptr;          // caller's beta_out
    double* U = nullptr;           // [max_steps+1][N*n_pad]
    double* V = nullptr;           // [max_steps+1][2N]
    double* WH = nullptr;          // [max_steps+1][2N]
    int32_t basis_cap = 0;
    int32_t nbasis = 0;
    bool ls_kappa_only = false;    // LSQR over the kt block only (step 0 of Sec. 5), fixed at init
    bool reorth_on = false;        // reorthogonalisation state fixed at qpat_lsqr_init
    double* coef = nullptr;        // [max_steps+1] Gram-Schmidt coefficients
    qpat::LsqrScal* ls = nullptr;
    qpat::LsqrScal* ls_host = nullptr;

    // reductions
    double* red_partials = nullptr;  // [kMaxRed]
    double* red_out = nullptr;       // [64]
    uint32_t* red_counter = nullptr;
    double* red_host = nullptr;      // pinned [64]

    int32_t* dev_flag = nullptr;     // error flag written by validation kernels

    // per-launch timing of the PCG iteration kernels
    bool prof_on = false;
    qpat_kstat prof[QPAT_NKSTAT]{};
    std::vector<hipEvent_t> ev_pool;

    // learned initial guess (conv net on the node lattice)
    qpat::GuessNet* guess = nullptr;

    // multigrid hierarchies of M_delta and K (lattice meshes)
    qpat::MgState* mg = nullptr;
    qpat::MgState* mgk = nullptr;

    // resident blocks per kernel configuration (occupancy x compute units)
    std::map<int, int> occupancy;
    std::map<std::string, int> st_occ;   // stencil kernel, keyed by kernel and LDS size

    // captured graphs of PCG iteration chunks, keyed by kernel configuration
    hipStream_t cap_stream = nullptr;
    std::map<std::string, hipGraphExec_t> graphs;

    std::vector<void*> allocs;
};

namespace qpat {

// ---- allocation / error helpers (api.hip)
qpat_status fail(qpat_ctx* c, qpat_status st, const char* fmt, ...);
qpat_status hip_check(qpat_ctx* c, hipError_t e, const char* what);
template <typename T>
qpat_status dalloc(qpat_ctx* c, T** p, size_t n) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, n * sizeof(T) > 0 ? n * sizeof(T) : 16);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, QPAT_ERR_OOM, "hipMalloc(%zu bytes) failed: %s", n * sizeof(T), hipGetErrorString(e));
    }
    c->allocs.push_back(q);
    *p = static_cast<T*>(q);
    return QPAT_OK;
}
qpat_status dfree(qpat_ctx* c, void* p);

#define QPAT_TRY(expr)                    \
    do {                                  \
        qpat_status _s = (expr);          \
        if (_s != QPAT_OK) return _s;     \
    } while (0)
#define QPAT_HIP(c, expr) QPAT_TRY(::qpat::hip_check((c), (expr), #expr))

inline int grid_for(int64_t items, int per_block, int cap) {
    int64_t g = (items + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<int>(g);
}

// ---- mesh.hip
qpat_status mesh_build(qpat_ctx* c, const double* coords, const int32_t* tets_in,
                       const int32_t* bfaces_in);

// ---- assemble.hip
qpat_status assemble_K(qpat_ctx* c);
qpat_status assemble_prior(qpat_ctx* c, const double* kt, const double* mt, int kind, double T,
                           double q, double b_over_a, double delta);
qpat_status assemble_load(qpat_ctx* c, const double* phi_src);
qpat_status exp_params(qpat_ctx* c, double kappa0, double mu0, const double* beta);
qpat_status check_positive(qpat_ctx* c, const double* a, int64_t n, bool* ok);

// ---- pcg.hip
// Which operator a solve uses.
enum class Op { K, Prior };

// ---- lattice.hip
// Detects the lattice numbering after mesh_build; allocates the stencil arrays.
qpat_status lattice_setup(qpat_ctx* c, const double* coords);
// Copies the assembled sliced-ELL operator into its stencil arrays.
qpat_status lattice_convert(qpat_ctx* c, Op op);
struct SolveStats {
    int32_t n_solves = 0, iters_max = 0, updates = 0;
    int64_t iters_sum = 0;
    double relres_max = 0.0;
    bool noconv = false;
    // per system solved, in order (block by block, right-hand side by right-hand side)
    std::vector<int32_t> rhs_iters;
    std::vector<double> rhs_relres;
    void add(int32_t iters, double relres, int32_t upd, bool done) {
        n_solves += 1;
        iters_max = std::max(iters_max, iters);
        iters_sum += iters;
        updates += upd;
        relres_max = std::max(relres_max, relres);
        if (!done) noconv = true;
        rhs_iters.push_back(iters);
        rhs_relres.push_back(relres);
    }
    void merge(const SolveStats& o) {
        n_solves += o.n_solves;
        iters_max = std::max(iters_max, o.iters_max);
        iters_sum += o.iters_sum;
        updates += o.updates;
        relres_max = std::max(relres_max, o.relres_max);
        noconv = noconv || o.noconv;
        rhs_iters.insert(rhs_iters.end(), o.rhs_iters.begin(), o.rhs_iters.end());
        rhs_relres.insert(rhs_relres.end(), o.rhs_relres.begin(), o.rhs_relres.end());
    }
};
// Solve op * x = b for B right-hand sides (interleaved [N][B], b in c->b64,
// result in c->x64). For Op::Prior, nsys = 2 systems with B = 1 ([2][N]).
// has_x0: c->x64 already holds the initial guess (K solves only)
qpat_status pcg_solve(qpat_ctx* c, Op op, int B, SolveStats* st, bool has_x0 = false);
qpat_status spmv64(qpat_ctx* c, Op op, int B, const double* x, double* y, double shift);

// ---- jacobian.hip
qpat_status forward_solve(qpat_ctx* c, SolveStats* st);
// J s: s [2N]; mode 0 -> out [n_ill][N]; mode 1 (LSQR) -> q = W (J s) - alpha u
qpat_status jvp_core(qpat_ctx* c, const double* s, int mode, double* out, SolveStats* st);
// J^T t: mode 0 -> t [n_ill][N]; mode 1 (LSQR) -> t = W u (interleaved), out = J^T t - beta what
qpat_status vjp_core(qpat_ctx* c, const double* t, int mode, double* out, SolveStats* st);

// ---- guess.hip
qpat_status guess_setup(qpat_ctx* c, int nx, int ny, int nz);
qpat_status guess_set_params(qpat_ctx* c, const float* p);
qpat_status guess_get_params(qpat_ctx* c, float* p);
qpat_status guess_eval_raw(qpat_ctx* c, const float* in, float* out);
qpat_status guess_grad_raw(qpat_ctx* c, const float* in, const float* target, float* grad, double* loss);
qpat_status guess_train_raw(qpat_ctx* c, const float* in, const float* target, float lr, double* loss);
qpat_status guess_train(qpat_ctx* c, const double* kappa, const double* mu, double k0, double m0,
                        const double* phih, const double* phi, float lr, double* loss);
qpat_status guess_fluence(qpat_ctx* c, const double* kappa, const double* mu, double k0, double m0,
                          const double* phih, double* phi0);
void guess_destroy(qpat_ctx* c);
qpat_status forward_solve_x0(qpat_ctx* c, const double* x0, SolveStats* st);

// ---- mg.hip
// The multigrid-preconditioned PCG for op: wanted by the options and possible
// on this mesh (lattice numbering, stencil form).
bool mg_available(const qpat_ctx* c, Op op);
// available and its hierarchy built
bool mg_ready(qpat_ctx* c, Op op);
// (Re)builds op's hierarchy from its current stencil arrays; no-op when unavailable.
qpat_status mg_setup(qpat_ctx* c, Op op);
// The same contract as pcg_solve (b in c->b64, x in c->x64, has_x0 for K).
qpat_status mg_solve(qpat_ctx* c, Op op, int B, SolveStats* st, bool has_x0 = false);
void mg_destroy(qpat_ctx* c);
// out [N][B] = scale U in for a Kuhn stencil form U [N][8] and in [N][ld]
// (columns col ... col + B - 1), LDS-tiled; *done = false when that path is
// not available (no current K hierarchy, B < 8, offsets past 32 bits).
// the tile schedule of the K hierarchy for blocks of B (qpat_tile_schedule)
qpat_status mg_tile_schedule(const qpat_ctx* c, int B, int32_t out[8]);
qpat_status mg_stencil_apply(qpat_ctx* c, int B, const double* U, const double* in, int ld, int col, double* out,
                             double scale, bool* done);

// ---- lsqr.hip
qpat_status dot(qpat_ctx* c, const double* a, const double* b, int64_t n, double* dev_out);
qpat_status lsqr_init_core(qpat_ctx* c, const double* chi, const double* w, const double* beta_lin);
qpat_status lsqr_step_core(qpat_ctx* c, SolveStats* st);
qpat_status misfit_core(qpat_ctx* c, const double* chi, const double* w, double* out);
// the file-scope scratch of the allocation-free misfit: its device address for
// c->device (looked up once per device; the device must be current)
qpat_status scratch_setup(qpat_ctx* c);
// ||W (chi - h)|| into out_dev[0] (device) with the partial sums in that scratch
qpat_status misfit_noalloc_core(qpat_ctx* c, const double* chi, const double* w, double* out_dev);
qpat_status init_guess_core(qpat_ctx* c, const double* chi, double mu0, double* beta_out);
// Gauss-Newton sums of the background fit: with r = W (chi - h) and the
// whitened columns W j1, W j2 ([n_ill][N], scaled in place), out[0..5] =
// (Wj1.Wj1, Wj1.Wj2, Wj2.Wj2, Wj1.r, Wj2.r, r.r) on the host.
qpat_status fit_sums(qpat_ctx* c, const double* chi, const double* w, double* j1, double* j2, double* rr,
                     double out[6]);
// zero [n] doubles on the context's stream (a kernel, not a memset node)
qpat_status zero_fill(qpat_ctx* c, double* p, int64_t n);
qpat_status prior_apply_core(qpat_ctx* c, const double* x, double* y);
qpat_status prior_solve_core(qpat_ctx* c, const double* p, double* r, SolveStats* st);

}  // namespace qpat
