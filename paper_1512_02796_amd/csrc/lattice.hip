// Stencil (lattice) form of the P1 operators on lexicographically numbered
// lattice meshes, such as the Kuhn voxel meshes of Sec. 5.
//
// Detection is combinatorial: the node numbering fixes candidate lattice
// dimensions (nx from the first change of the y or z coordinate, nx ny from
// the first change of z), and the form is used only if every entry of the
// sliced-ELL pattern joins nodes at most one lattice step apart along each
// axis. The coordinates never enter the operator, so a positive check makes
// the stencil product equal to the sliced-ELL one up to the order of the sum.
#include "qpat_internal.h"

namespace qpat {
namespace {

__global__ void k_first_change(const double* __restrict__ coords, int64_t N, int64_t* out) {
    __shared__ int64_t s_row, s_plane;
    if (threadIdx.x == 0) {
        s_row = N;
        s_plane = N;
    }
    __syncthreads();
    const double y0 = coords[1], z0 = coords[2];
    int64_t row = N, plane = N;
    for (int64_t i = 1 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double y = coords[3 * i + 1], z = coords[3 * i + 2];
        if (z != z0) plane = i < plane ? i : plane;
        if (z != z0 || y != y0) row = i < row ? i : row;
    }
    atomicMin(reinterpret_cast<unsigned long long*>(&s_row), static_cast<unsigned long long>(row));
    atomicMin(reinterpret_cast<unsigned long long*>(&s_plane), static_cast<unsigned long long>(plane));
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMin(reinterpret_cast<unsigned long long*>(out), static_cast<unsigned long long>(s_row));
        atomicMin(reinterpret_cast<unsigned long long*>(out + 1), static_cast<unsigned long long>(s_plane));
    }
}

// bit (dx+1) + 3 (dy+1) + 9 (dz+1) of out[0] for every offset in the pattern;
// out[1] = 1 if some entry is more than one lattice step away
__global__ void k_offsets(Sell s, int64_t N, int32_t nx, int32_t ny, uint32_t* out) {
    __shared__ uint32_t s_mask, s_far;
    if (threadIdx.x == 0) {
        s_mask = 0;
        s_far = 0;
    }
    __syncthreads();
    uint32_t mask = 0, far = 0;
    const int64_t nxy = (int64_t)nx * ny;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
        const int32_t base = s.slice_ptr[i / kSlice] + static_cast<int32_t>(i % kSlice);
        const int32_t n = s.rowlen[i];
        for (int32_t j = 0; j < n; ++j) {
            const int64_t col = s.cols[base + j * kSlice];
            const int64_t dx = col % nx - ix, dy = (col / nx) % ny - iy, dz = col / nxy - iz;
            if (dx < -1 || dx > 1 || dy < -1 || dy > 1 || dz < -1 || dz > 1)
                far = 1;
            else
                mask |= 1u << ((dx + 1) + 3 * (dy + 1) + 9 * (dz + 1));
        }
    }
    atomicOr(&s_mask, mask);
    atomicOr(&s_far, far);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicOr(out, s_mask);
        atomicOr(out + 1, s_far);
    }
}

// U[sys][i][code[offset]] = A_sys(i, col) for the diagonal and upper entries of row i
__global__ void k_to_lattice(Sell s, int64_t N, Lattice lat, const double* __restrict__ vals, int64_t vals_stride,
                             double* __restrict__ u64, float* __restrict__ u32) {
    const int32_t sys = blockIdx.y;
    const double* __restrict__ v = vals + sys * vals_stride;
    const int64_t nxy = (int64_t)lat.nx * lat.ny;
    const int64_t M1 = lat.m + 1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ix = i % lat.nx, iy = (i / lat.nx) % lat.ny, iz = i / nxy;
        const int32_t base = s.slice_ptr[i / kSlice] + static_cast<int32_t>(i % kSlice);
        const int32_t n = s.rowlen[i];
        for (int32_t j = 0; j < n; ++j) {
            const int32_t e = base + j * kSlice;
            const int64_t col = s.cols[e];
            const int64_t dx = col % lat.nx - ix, dy = (col / lat.nx) % lat.ny - iy, dz = col / nxy - iz;
            const int c = lat.code[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];
            if (c < 0) continue;
            const int64_t at = (sys * N + i) * M1 + c;   // [sys][node][m+1]
            if (u64) u64[at] = v[e];
            if (u32) u32[at] = static_cast<float>(v[e]);
        }
    }
}

}  // namespace

qpat_status lattice_setup(qpat_ctx* c, const double* coords) {
    Lattice& L = c->lat;
    L = Lattice{};
    const int64_t N = c->N;
    int64_t* d64 = nullptr;
    QPAT_TRY(dalloc(c, &d64, 4));
    int64_t init[2] = {N, N};
    QPAT_HIP(c, hipMemcpyAsync(d64, init, sizeof init, hipMemcpyHostToDevice, c->stream));
    hipLaunchKernelGGL(k_first_change, dim3(grid_for(N, kThreads, 2048)), dim3(kThreads), 0, c->stream, coords, N,
                       d64);
    int64_t first[2];
    QPAT_HIP(c, hipMemcpyAsync(first, d64, sizeof first, hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    QPAT_TRY(dfree(c, d64));
    const int64_t nx = first[0], nxy = first[1];
    if (nx < 2 || nxy <= nx || nxy % nx != 0 || N % nxy != 0 || N / nxy < 2) return QPAT_OK;
    if (nx > (1 << 30) || nxy / nx > (1 << 30) || N / nxy > (1 << 30)) return QPAT_OK;
    const int32_t ny = static_cast<int32_t>(nxy / nx), nz = static_cast<int32_t>(N / nxy);

    uint32_t* d32 = nullptr;
    QPAT_TRY(dalloc(c, &d32, 2));
    QPAT_HIP(c, hipMemsetAsync(d32, 0, 2 * sizeof(uint32_t), c->stream));
    hipLaunchKernelGGL(k_offsets, dim3(grid_for(N, kThreads, 2048)), dim3(kThreads), 0, c->stream, c->sell, N,
                       static_cast<int32_t>(nx), ny, d32);
    uint32_t res[2];
    QPAT_HIP(c, hipMemcpyAsync(res, d32, sizeof res, hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    QPAT_TRY(dfree(c, d32));
    if (res[1] != 0) return QPAT_OK;
    const uint32_t mask = res[0];
    if (!((mask >> 13) & 1u)) return QPAT_OK;   // no diagonal: not a pattern this library builds
    for (int code = 0; code < 27; ++code)       // a node-node pattern is symmetric
        if (((mask >> code) & 1u) != ((mask >> (26 - code)) & 1u)) return QPAT_OK;

    Lattice lat;
    lat.nx = static_cast<int32_t>(nx);
    lat.ny = ny;
    lat.nz = nz;
    for (int code = 0; code < 27; ++code) lat.code[code] = -1;
    lat.code[13] = 0;
    for (int code = 14; code < 27; ++code) {
        if (!((mask >> code) & 1u)) continue;
        const int j = ++lat.m;
        lat.dx[j - 1] = static_cast<int8_t>(code % 3 - 1);
        lat.dy[j - 1] = static_cast<int8_t>((code / 3) % 3 - 1);
        lat.dz[j - 1] = static_cast<int8_t>(code / 9 - 1);
        lat.code[code] = static_cast<int8_t>(j);
    }
    int32_t tab[4 * kMaxUpper] = {};
    for (int j = 0; j < lat.m; ++j) {
        tab[4 * j] = lat.dx[j];
        tab[4 * j + 1] = lat.dy[j];
        tab[4 * j + 2] = lat.dz[j];
        tab[4 * j + 3] = lat.dx[j] + lat.nx * (lat.dy[j] + ny * lat.dz[j]);
    }
    QPAT_TRY(dalloc(c, &c->lat_tab, 4 * kMaxUpper));
    QPAT_HIP(c, hipMemcpyAsync(c->lat_tab, tab, sizeof tab, hipMemcpyHostToDevice, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    const int64_t U = (int64_t)(lat.m + 1) * N;
    QPAT_TRY(dalloc(c, &c->KU64, U));
    QPAT_TRY(dalloc(c, &c->KU32, U));
    QPAT_TRY(dalloc(c, &c->MU64, 2 * U));
    // entries outside the pattern stay zero for the life of the context
    QPAT_HIP(c, hipMemsetAsync(c->KU64, 0, U * sizeof(double), c->stream));
    QPAT_HIP(c, hipMemsetAsync(c->KU32, 0, U * sizeof(float), c->stream));
    QPAT_HIP(c, hipMemsetAsync(c->MU64, 0, 2 * U * sizeof(double), c->stream));
    lat.on = true;
    L = lat;
    // the Kuhn pattern with equal voxels: spacings from nodes 0, 1, nx and nx ny
    // (the voxel form of the Jacobian kernels is checked against the element
    // form before its first use)
    c->vox = -1;
    if (lat.m == 7) {
        double p[4][3];
        const int64_t at[4] = {0, 1, nx, nxy};
        for (int q = 0; q < 4; ++q)
            QPAT_HIP(c, hipMemcpyAsync(p[q], coords + 3 * at[q], 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        QPAT_HIP(c, hipStreamSynchronize(c->stream));
        c->vox_h[0] = p[1][0] - p[0][0];
        c->vox_h[1] = p[2][1] - p[0][1];
        c->vox_h[2] = p[3][2] - p[0][2];
        if (c->vox_h[0] > 0.0 && c->vox_h[1] > 0.0 && c->vox_h[2] > 0.0) c->vox = 0;
    }
    return QPAT_OK;
}

qpat_status lattice_convert(qpat_ctx* c, Op op) {
    if (!c->lat.on) return QPAT_OK;
    const int g = grid_for(c->N, kThreads, 8192);
    if (op == Op::K)
        hipLaunchKernelGGL(k_to_lattice, dim3(g, 1), dim3(kThreads), 0, c->stream, c->sell, c->N, c->lat, c->K64,
                           (int64_t)0, c->KU64, c->KU32);
    else
        hipLaunchKernelGGL(k_to_lattice, dim3(g, 2), dim3(kThreads), 0, c->stream, c->sell, c->N, c->lat, c->M64,
                           (int64_t)c->sell.len, c->MU64, static_cast<float*>(nullptr));
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

}  // namespace qpat
