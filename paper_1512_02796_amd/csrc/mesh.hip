// Mesh setup on the device: element geometry, node->element adjacency and the
// sliced-ELL sparsity pattern of the P1 system matrix.
//
// P1 basis on a tetrahedral partition (Sec. 3, eq. (3.2)); every FEM matrix
// of the path (K, the load operators G(1), G(2), the prior M) lives on the
// node-node pattern of that partition.
#include <cstring>

#include "qpat_internal.h"

namespace qpat {
namespace {

enum : int32_t {
    kFlagIndex = 1,
    kFlagDegenerate = 2,
    kFlagRowTooLong = 4,
    kFlagFaceDegenerate = 8,
    kFlagIsolated = 16,
    kFlagBadFace = 32
};

__global__ void k_check_index(const int32_t* idx, int64_t n, int64_t N, int32_t* flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = idx[i];
        if (v < 0 || v >= N) atomicOr(flag, kFlagIndex);
    }
}

// |T| and the gradients of the barycentric coordinates l1, l2, l3 (l0 = 1 - l1 - l2 - l3).
// With edge rows a = x1 - x0, b = x2 - x0, c = x3 - x0 and det = a.(b x c):
// grad l1 = (b x c)/det, grad l2 = (c x a)/det, grad l3 = (a x b)/det.
__global__ void k_geometry(const double* __restrict__ X, const int32_t* __restrict__ tets, int64_t E,
                           double* __restrict__ geo, int32_t* flag) {
    int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; e < E; e += (int64_t)gridDim.x * blockDim.x) {
        int32_t v0 = tets[4 * e], v1 = tets[4 * e + 1], v2 = tets[4 * e + 2], v3 = tets[4 * e + 3];
        double x0 = X[3 * v0], y0 = X[3 * v0 + 1], z0 = X[3 * v0 + 2];
        double ax = X[3 * v1] - x0, ay = X[3 * v1 + 1] - y0, az = X[3 * v1 + 2] - z0;
        double bx = X[3 * v2] - x0, by = X[3 * v2 + 1] - y0, bz = X[3 * v2 + 2] - z0;
        double cx = X[3 * v3] - x0, cy = X[3 * v3 + 1] - y0, cz = X[3 * v3 + 2] - z0;
        double bcx = by * cz - bz * cy, bcy = bz * cx - bx * cz, bcz = bx * cy - by * cx;
        double cax = cy * az - cz * ay, cay = cz * ax - cx * az, caz = cx * ay - cy * ax;
        double abx = ay * bz - az * by, aby = az * bx - ax * bz, abz = ax * by - ay * bx;
        double det = ax * bcx + ay * bcy + az * bcz;
        double la = fmax(fmax(fabs(ax), fabs(ay)), fabs(az));
        double lb = fmax(fmax(fabs(bx), fabs(by)), fabs(bz));
        double lc = fmax(fmax(fabs(cx), fabs(cy)), fabs(cz));
        double lm = fmax(fmax(la, lb), lc);
        double* g = geo + kTetGeo * e;
        if (!(fabs(det) > 1e-12 * lm * lm * lm)) {
            atomicOr(flag, kFlagDegenerate);
            for (int k = 0; k < kTetGeo; ++k) g[k] = 0.0;
            continue;
        }
        double inv = 1.0 / det;
        g[0] = fabs(det) / 6.0;
        g[1] = bcx * inv; g[2] = bcy * inv; g[3] = bcz * inv;
        g[4] = cax * inv; g[5] = cay * inv; g[6] = caz * inv;
        g[7] = abx * inv; g[8] = aby * inv; g[9] = abz * inv;
        g[10] = 0.0; g[11] = 0.0;
    }
}

// geometry class of each tetrahedron: the first of the K candidates whose
// kTetGeo doubles equal its own bit for bit; a tetrahedron matching none sets
// *flag (then the classes are not used)
__global__ void k_geo_classify(const double* __restrict__ geo, int64_t E, const double* __restrict__ cand, int K,
                               uint8_t* __restrict__ cls, int32_t* flag) {
    for (int64_t e = blockIdx.x * (int64_t)kThreads + threadIdx.x; e < E; e += (int64_t)gridDim.x * kThreads) {
        const unsigned long long* g = reinterpret_cast<const unsigned long long*>(geo + kTetGeo * e);
        int found = -1;
        for (int k = 0; k < K && found < 0; ++k) {
            const unsigned long long* c = reinterpret_cast<const unsigned long long*>(cand + kTetGeo * k);
            bool same = true;
#pragma unroll
            for (int d = 0; d < kTetGeo; ++d) same = same && g[d] == c[d];
            if (same) found = k;
        }
        if (found < 0) {
            *flag = 1;
            cls[e] = 0;
        } else {
            cls[e] = static_cast<uint8_t>(found);
        }
    }
}

__global__ void k_face_area(const double* __restrict__ X, const int32_t* __restrict__ f, int64_t F,
                            double* __restrict__ area, int32_t* flag) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < F; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v0 = f[3 * i], v1 = f[3 * i + 1], v2 = f[3 * i + 2];
        double ax = X[3 * v1] - X[3 * v0], ay = X[3 * v1 + 1] - X[3 * v0 + 1], az = X[3 * v1 + 2] - X[3 * v0 + 2];
        double bx = X[3 * v2] - X[3 * v0], by = X[3 * v2 + 1] - X[3 * v0 + 1], bz = X[3 * v2 + 2] - X[3 * v0 + 2];
        double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        double a = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
        double lm = fmax(fmax(fabs(ax), fabs(ay)), fmax(fmax(fabs(az), fabs(bx)), fmax(fabs(by), fabs(bz))));
        if (!(a > 1e-12 * lm * lm)) atomicOr(flag, kFlagFaceDegenerate);
        area[i] = a;
    }
}

// count[v] += 1 for every (element, local vertex) incidence
__global__ void k_count(const int32_t* __restrict__ conn, int64_t n, int32_t* __restrict__ cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) atomicAdd(&cnt[conn[i]], 1);
}

// adjacency entry i (= element * k + local vertex) appended to node conn[i]'s list
__global__ void k_fill(const int32_t* __restrict__ conn, int64_t n, const int32_t* __restrict__ ptr,
                       int32_t* __restrict__ cursor, int32_t* __restrict__ adj) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        int32_t v = conn[i];
        int32_t pos = atomicAdd(&cursor[v], 1);
        adj[ptr[v] + pos] = static_cast<int32_t>(i);
    }
}

// sort each node's adjacency list so that every later sweep is deterministic
__global__ void k_sort_lists(const int32_t* __restrict__ ptr, int32_t* __restrict__ adj, int64_t N) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; v < N; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t b = ptr[v], e = ptr[v + 1];
        for (int32_t i = b + 1; i < e; ++i) {
            int32_t key = adj[i];
            int32_t j = i - 1;
            while (j >= b && adj[j] > key) {
                adj[j + 1] = adj[j];
                --j;
            }
            adj[j + 1] = key;
        }
    }
}

// Sorted unique neighbour list of every node (itself included) into tmp[N][kMaxRow].
__global__ void k_row_pattern(const int32_t* __restrict__ tets, const int32_t* __restrict__ n2t_ptr,
                              const int32_t* __restrict__ n2t, int64_t N, int32_t* __restrict__ tmp,
                              int32_t* __restrict__ rowlen, int32_t* flag) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; v < N; v += (int64_t)gridDim.x * blockDim.x) {
        int32_t* lst = tmp + v * kMaxRow;
        int32_t n = 0;
        bool over = false;
        for (int32_t q = n2t_ptr[v]; q < n2t_ptr[v + 1] && !over; ++q) {
            int32_t e = n2t[q] >> 2;
            for (int b = 0; b < 4; ++b) {
                int32_t j = tets[4 * e + b];
                int32_t pos = 0;
                while (pos < n && lst[pos] < j) ++pos;
                if (pos < n && lst[pos] == j) continue;
                if (n == kMaxRow) {
                    over = true;
                    break;
                }
                for (int32_t m = n; m > pos; --m) lst[m] = lst[m - 1];
                lst[pos] = j;
                ++n;
            }
        }
        if (over) atomicOr(flag, kFlagRowTooLong);
        if (n == 0) atomicOr(flag, kFlagIsolated);
        rowlen[v] = n;
    }
}

// every edge of a boundary triangle must be an edge of the tetrahedral mesh
__global__ void k_check_bfaces(const int32_t* __restrict__ bf, int64_t F, const int32_t* __restrict__ tmp,
                               const int32_t* __restrict__ rowlen, int32_t* flag) {
    int64_t f = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    for (; f < F; f += (int64_t)gridDim.x * blockDim.x) {
        for (int a = 0; a < 3; ++a) {
            const int32_t i = bf[3 * f + a], j = bf[3 * f + (a + 1) % 3];
            const int32_t* lst = tmp + (int64_t)i * kMaxRow;
            bool found = false;
            for (int32_t k = 0; k < rowlen[i]; ++k) found |= lst[k] == j;
            if (!found) atomicOr(flag, kFlagBadFace);
        }
    }
}

__global__ void k_slice_width(const int32_t* __restrict__ rowlen, int64_t N, int32_t nslices,
                              int32_t* __restrict__ slice_w, int32_t* __restrict__ slice_len) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslices) return;
    int32_t w = 0;
    for (int k = 0; k < kSlice; ++k) {
        int64_t r = (int64_t)s * kSlice + k;
        if (r < N) w = max(w, rowlen[r]);
    }
    slice_w[s] = w;
    slice_len[s] = w * kSlice;
}

// thread per (row, k < slice width): scatter the pattern into the sliced layout
__global__ void k_fill_sell(const int32_t* __restrict__ tmp, const int32_t* __restrict__ rowlen,
                            const int32_t* __restrict__ slice_ptr, const int32_t* __restrict__ slice_w,
                            int64_t N, int32_t nslices, int32_t* __restrict__ cols, int32_t* __restrict__ diag) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t total = (int64_t)nslices * kSlice;
    for (; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int64_t row = t;
        int32_t s = static_cast<int32_t>(row / kSlice);
        int32_t lane = static_cast<int32_t>(row % kSlice);
        int32_t w = slice_w[s];
        int32_t base = slice_ptr[s] + lane;
        if (row >= N) {
            for (int k = 0; k < w; ++k) cols[base + k * kSlice] = 0;
            continue;
        }
        int32_t n = rowlen[row];
        const int32_t* lst = tmp + row * kMaxRow;
        for (int k = 0; k < w; ++k) {
            int32_t col = k < n ? lst[k] : static_cast<int32_t>(row);
            cols[base + k * kSlice] = col;
            if (k < n && col == row) diag[row] = k;
        }
    }
}

// Exclusive prefix sum (set-up only: adjacency offsets, slice offsets). A block
// scans a tile of kScanTile values -- each thread a run of kScanPer, then the
// thread totals in LDS -- and writes the tile's total; the totals are scanned
// the same way (recursively) and added back. Each block reads its whole tile
// before writing it, so `in` may alias `out`.
constexpr int kScanT = 256, kScanPer = 16, kScanTile = kScanT * kScanPer;

__global__ __launch_bounds__(kScanT) void k_scan_tile(const int32_t* in, int32_t* out, int64_t n,
                                                       int32_t* __restrict__ tile_sum) {
    __shared__ int32_t part[kScanT];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
    int32_t v[kScanPer];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        v[k] = base + k < n ? in[base + k] : 0;
        s += v[k];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < kScanT; off <<= 1) {   // inclusive scan of the thread totals
        const int32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = part[threadIdx.x] - s;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanT - 1) tile_sum[blockIdx.x] = part[kScanT - 1];
}

__global__ void k_scan_add(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ tile_off) {
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] += tile_off[i / kScanTile];
}

qpat_status exclusive_scan(qpat_ctx* c, const int32_t* in, int32_t* out, int64_t n) {
    if (n <= 0) return QPAT_OK;
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    int32_t *sum = nullptr, *off = nullptr;
    QPAT_TRY(dalloc(c, &sum, tiles));
    QPAT_TRY(dalloc(c, &off, tiles));
    hipLaunchKernelGGL(k_scan_tile, dim3(static_cast<uint32_t>(tiles)), dim3(kScanT), 0, c->stream, in, out, n, sum);
    if (tiles > 1) {
        QPAT_TRY(exclusive_scan(c, sum, off, tiles));
        hipLaunchKernelGGL(k_scan_add, dim3(static_cast<uint32_t>((n + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                           c->stream, out, n, off);
    }
    QPAT_HIP(c, hipGetLastError());
    QPAT_TRY(dfree(c, sum));   // hipFree waits for the kernels above
    QPAT_TRY(dfree(c, off));
    return QPAT_OK;
}

// adjacency of nodes to the k-vertex cells of conn [n_cells][k]
qpat_status build_adjacency(qpat_ctx* c, const int32_t* conn, int64_t n_entries, int32_t** ptr_out,
                            int32_t** adj_out) {
    const int64_t N = c->N;
    int32_t *cnt = nullptr, *ptr = nullptr, *adj = nullptr;
    QPAT_TRY(dalloc(c, &cnt, N + 1));
    QPAT_TRY(dalloc(c, &ptr, N + 1));
    QPAT_TRY(dalloc(c, &adj, n_entries));
    QPAT_HIP(c, hipMemsetAsync(cnt, 0, (N + 1) * sizeof(int32_t), c->stream));
    int g = grid_for(n_entries, kThreads, 65536);
    if (n_entries > 0) hipLaunchKernelGGL(k_count, dim3(g), dim3(kThreads), 0, c->stream, conn, n_entries, cnt);
    QPAT_TRY(exclusive_scan(c, cnt, ptr, N + 1));
    QPAT_HIP(c, hipMemsetAsync(cnt, 0, (N + 1) * sizeof(int32_t), c->stream));
    if (n_entries > 0) hipLaunchKernelGGL(k_fill, dim3(g), dim3(kThreads), 0, c->stream, conn, n_entries, ptr, cnt, adj);
    hipLaunchKernelGGL(k_sort_lists, dim3(grid_for(N, kThreads, 65536)), dim3(kThreads), 0, c->stream, ptr, adj, N);
    QPAT_HIP(c, hipGetLastError());
    QPAT_TRY(dfree(c, cnt));
    *ptr_out = ptr;
    *adj_out = adj;
    return QPAT_OK;
}

qpat_status read_flag(qpat_ctx* c, int32_t* out) {
    QPAT_HIP(c, hipMemcpyAsync(out, c->dev_flag, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    return QPAT_OK;
}

// Geometry classes (see qpat_ctx::geo_cls): candidates are the distinct
// geometries among the first kGeoProbe tetrahedra; every tetrahedron must
// match one of at most kGeoMaxCls of them bit for bit, else no classes.
constexpr int kGeoProbe = 64, kGeoMaxCls = 16;
qpat_status classify_geometry(qpat_ctx* c) {
    const int64_t E = c->E;
    const int probe = static_cast<int>(std::min<int64_t>(E, kGeoProbe));
    std::vector<double> first(static_cast<size_t>(probe) * kTetGeo);
    QPAT_HIP(c, hipMemcpyAsync(first.data(), c->geo, first.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    std::vector<double> cand;
    for (int e = 0; e < probe; ++e) {
        const double* g = first.data() + static_cast<size_t>(e) * kTetGeo;
        bool seen = false;
        for (size_t k = 0; k < cand.size() / kTetGeo && !seen; ++k)
            seen = std::memcmp(cand.data() + k * kTetGeo, g, kTetGeo * sizeof(double)) == 0;
        if (!seen) cand.insert(cand.end(), g, g + kTetGeo);
    }
    const int K = static_cast<int>(cand.size() / kTetGeo);
    if (K == 0 || K > kGeoMaxCls) return QPAT_OK;
    double* tab = nullptr;
    uint8_t* cls = nullptr;
    int32_t* miss = nullptr;   // its own flag: the mesh checks share dev_flag
    QPAT_TRY(dalloc(c, &tab, cand.size()));
    QPAT_TRY(dalloc(c, &cls, E));
    QPAT_TRY(dalloc(c, &miss, 1));
    QPAT_HIP(c, hipMemcpyAsync(tab, cand.data(), cand.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
    QPAT_HIP(c, hipMemsetAsync(miss, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_geo_classify, dim3(grid_for(E, kThreads, 65536)), dim3(kThreads), 0, c->stream, c->geo, E,
                       tab, K, cls, miss);
    QPAT_HIP(c, hipGetLastError());
    int32_t flag = 0;
    QPAT_HIP(c, hipMemcpyAsync(&flag, miss, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    QPAT_TRY(dfree(c, miss));
    if (flag) {
        QPAT_TRY(dfree(c, cls));
        QPAT_TRY(dfree(c, tab));
        return QPAT_OK;
    }
    c->geo_cls = cls;
    c->geo_tab = tab;
    c->geo_ncls = K;
    return QPAT_OK;
}

}  // namespace

qpat_status mesh_build(qpat_ctx* c, const double* coords, const int32_t* tets_in, const int32_t* bfaces_in) {
    const int64_t N = c->N, E = c->E, F = c->Fb;
    if (4 * E >= (int64_t(1) << 31) || 3 * F >= (int64_t(1) << 31) || N * (int64_t)kMaxRow >= (int64_t(1) << 40))
        return fail(c, QPAT_ERR_ARG, "mesh too large for 32-bit adjacency indices");
    QPAT_TRY(dalloc(c, &c->dev_flag, 4));
    QPAT_HIP(c, hipMemsetAsync(c->dev_flag, 0, 4 * sizeof(int32_t), c->stream));

    QPAT_TRY(dalloc(c, &c->tets, 4 * E));
    QPAT_HIP(c, hipMemcpyAsync(c->tets, tets_in, 4 * E * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));
    QPAT_TRY(dalloc(c, &c->bfaces, 3 * F));
    if (F > 0)
        QPAT_HIP(c, hipMemcpyAsync(c->bfaces, bfaces_in, 3 * F * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream));

    hipLaunchKernelGGL(k_check_index, dim3(grid_for(4 * E, kThreads, 16384)), dim3(kThreads), 0, c->stream,
                       c->tets, 4 * E, N, c->dev_flag);
    if (F > 0)
        hipLaunchKernelGGL(k_check_index, dim3(grid_for(3 * F, kThreads, 16384)), dim3(kThreads), 0, c->stream,
                           c->bfaces, 3 * F, N, c->dev_flag);
    int32_t flag = 0;
    QPAT_TRY(read_flag(c, &flag));
    if (flag & kFlagIndex) return fail(c, QPAT_ERR_MESH, "node index out of range in tets or bfaces");

    QPAT_TRY(dalloc(c, &c->geo, kTetGeo * E));
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(E, kThreads, 65536)), dim3(kThreads), 0, c->stream, coords, c->tets,
                       E, c->geo, c->dev_flag);
    QPAT_TRY(dalloc(c, &c->barea, F));
    if (F > 0)
        hipLaunchKernelGGL(k_face_area, dim3(grid_for(F, kThreads, 65536)), dim3(kThreads), 0, c->stream, coords,
                           c->bfaces, F, c->barea, c->dev_flag);
    QPAT_TRY(read_flag(c, &flag));
    if (flag & kFlagDegenerate) return fail(c, QPAT_ERR_MESH, "degenerate (zero-volume) tetrahedron");
    if (flag & kFlagFaceDegenerate) return fail(c, QPAT_ERR_MESH, "degenerate boundary triangle");

    QPAT_TRY(classify_geometry(c));
    QPAT_TRY(build_adjacency(c, c->tets, 4 * E, &c->n2t_ptr, &c->n2t));
    QPAT_TRY(build_adjacency(c, c->bfaces, 3 * F, &c->n2f_ptr, &c->n2f));

    // row pattern
    Sell& s = c->sell;
    s.N = N;
    s.nslices = static_cast<int32_t>((N + kSlice - 1) / kSlice);
    int32_t* tmp = nullptr;
    QPAT_TRY(dalloc(c, &tmp, N * kMaxRow));
    QPAT_TRY(dalloc(c, &s.rowlen, N));
    hipLaunchKernelGGL(k_row_pattern, dim3(grid_for(N, kThreads, 65536)), dim3(kThreads), 0, c->stream, c->tets,
                       c->n2t_ptr, c->n2t, N, tmp, s.rowlen, c->dev_flag);
    if (F > 0)
        hipLaunchKernelGGL(k_check_bfaces, dim3(grid_for(F, kThreads, 65536)), dim3(kThreads), 0, c->stream,
                           c->bfaces, F, tmp, s.rowlen, c->dev_flag);
    QPAT_TRY(read_flag(c, &flag));
    if (flag & kFlagRowTooLong) return fail(c, QPAT_ERR_MESH, "a node has more than %d neighbours", kMaxRow - 1);
    if (flag & kFlagIsolated) return fail(c, QPAT_ERR_MESH, "a node belongs to no tetrahedron");
    if (flag & kFlagBadFace) return fail(c, QPAT_ERR_MESH, "a boundary triangle is not a face of the mesh");

    int32_t* slice_len = nullptr;
    QPAT_TRY(dalloc(c, &s.slice_w, s.nslices));
    QPAT_TRY(dalloc(c, &slice_len, s.nslices + 1));
    QPAT_TRY(dalloc(c, &s.slice_ptr, s.nslices + 1));
    QPAT_HIP(c, hipMemsetAsync(slice_len + s.nslices, 0, sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_slice_width, dim3(grid_for(s.nslices, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream,
                       s.rowlen, N, s.nslices, s.slice_w, slice_len);
    QPAT_TRY(exclusive_scan(c, slice_len, s.slice_ptr, s.nslices + 1));
    int32_t total = 0;
    QPAT_HIP(c, hipMemcpyAsync(&total, s.slice_ptr + s.nslices, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    s.len = total;
    QPAT_TRY(dalloc(c, &s.cols, s.len));
    QPAT_TRY(dalloc(c, &s.diag, N));
    QPAT_HIP(c, hipMemsetAsync(s.diag, 0, N * sizeof(int32_t), c->stream));
    hipLaunchKernelGGL(k_fill_sell, dim3(grid_for((int64_t)s.nslices * kSlice, kThreads, 65536)), dim3(kThreads), 0,
                       c->stream, tmp, s.rowlen, s.slice_ptr, s.slice_w, N, s.nslices, s.cols, s.diag);
    QPAT_HIP(c, hipGetLastError());
    // the widest slice bounds every per-row loop
    std::vector<int32_t> w(s.nslices);
    QPAT_HIP(c, hipMemcpyAsync(w.data(), s.slice_w, s.nslices * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    s.max_width = 0;
    for (int32_t v : w) s.max_width = v > s.max_width ? v : s.max_width;
    QPAT_TRY(dfree(c, tmp));
    QPAT_TRY(dfree(c, slice_len));
    return QPAT_OK;
}

}  // namespace qpat
