// Learned initial guess for the forward PCG solves: a four-layer 3x3x3
// convolutional network on the node lattice (channels 3 -> 16 -> 16 -> 16 -> 1,
// ReLU between layers, zero padding), BF16 weights and activations, FP32
// accumulation on MFMA, trained on the device.
//
// Inputs per illumination k (nodal): log(mu/mu0), log(kappa/kappa0) and
// log(phi_hom,k), the fluence of the homogeneous (kappa0, mu0) medium for that
// source. Output: the log correction, phi0 = phi_hom,k exp(net). The solve that
// starts from phi0 stops on the same ||b - K x|| <= rtol ||b|| as a zero start.
//
// Convolutions are implicit GEMMs on the 16x16x16 BF16 MFMA: a wavefront owns
// 16 consecutive lattice points x 16 output channels; the K dimension is one
// tap x 16 input channels (or four taps x 4 channels for the 3-channel input
// layer, padded to 4). Weight gradients are the same product with the voxel
// index as the K dimension, split over wavefronts and reduced in fixed order.
#include <cmath>

#include "qpat_internal.h"

namespace qpat {
namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kLayers = 4;
constexpr int kCin[kLayers] = {3, 16, 16, 16};
constexpr int kCout[kLayers] = {16, 16, 16, 1};
constexpr int kParams = 15601;

__host__ __device__ inline int param_offset(int layer) {
    int off = 0;
    for (int l = 0; l < layer; ++l) off += kCout[l] * kCin[l] * 27 + kCout[l];
    return off;
}

__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return static_cast<uint16_t>(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);                                              // round to nearest even
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float(static_cast<uint32_t>(b) << 16); }

struct Lat {
    int nx, ny, nz;
    int64_t V;
};

// neighbour of v through tap t ((dz, dy, dx) in {-1,0,1}^3, dx fastest); -1 outside
__device__ __forceinline__ int64_t neighbour(const Lat& L, int x, int y, int z, int t) {
    const int dx = t % 3 - 1, dy = (t / 3) % 3 - 1, dz = t / 9 - 1;
    const int xx = x + dx, yy = y + dy, zz = z + dz;
    if (xx < 0 || xx >= L.nx || yy < 0 || yy >= L.ny || zz < 0 || zz >= L.nz) return -1;
    return xx + (int64_t)L.nx * (yy + (int64_t)L.ny * zz);
}

// ---------------------------------------------------------------- forward / backward-data
// MODE 0: out bf16 [V][16] = relu(z + bias)
// MODE 1: out f32 [V]      = z[:, 0] + bias[0]
// MODE 2: out bf16 [V][16] = z * (mask[V][16] > 0)          (backward data; no bias)
template <int CIN, int MODE>
__global__ __launch_bounds__(kThreads) void k_conv(Lat L, const uint16_t* __restrict__ X,
                                                   const uint16_t* __restrict__ Wp, const float* __restrict__ bias,
                                                   const uint16_t* __restrict__ mask, void* __restrict__ out) {
    constexpr int NCH = CIN == 16 ? 27 : 7;
    __shared__ s4 wsh[NCH][64];
    for (int i = threadIdx.x; i < NCH * 64; i += kThreads) {
        const int m = i / 64, l = i % 64;
        wsh[m][l] = *reinterpret_cast<const s4*>(Wp + ((int64_t)m * 16 + l % 16) * 16 + 4 * (l / 16));
    }
    __syncthreads();
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16;
    const int64_t ntiles = (L.V + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += (int64_t)gridDim.x * 4) {
        const int64_t v = tile * 16 + lane % 16;
        const bool vok = v < L.V;
        const int x = static_cast<int>(v % L.nx);
        const int y = static_cast<int>((v / L.nx) % L.ny);
        const int z = static_cast<int>(v / ((int64_t)L.nx * L.ny));
        // every tap's A fragment first, then the chain of MFMAs: the loads
        // are in flight together instead of each waiting for the MFMA before
        // it. Buffer loads with 32-bit offsets (V CIN 2 < 2^31 bytes, checked
        // on the host); a tap outside the lattice reads 0 (offset kOut).
        const auto bx = rsrc(X, static_cast<uint32_t>(L.V * CIN * 2));
        auto tap = [&](int m) {
            const int t = CIN == 16 ? m : 4 * m + g;
            const int ci0 = CIN == 16 ? 4 * g : 0;
            const int64_t nb = vok && t < 27 ? neighbour(L, x, y, z, t) : -1;
            const uint32_t off = nb >= 0 ? static_cast<uint32_t>(nb * CIN + ci0) * 2u : kOut;
            return bload<s4>(bx, off);
        };
        f4 acc = {0.f, 0.f, 0.f, 0.f};
        // taps in groups of one z-plane (9), the loads of the next group issued
        // before the MFMAs of this one (a two-group pipeline keeps the
        // registers, and so the waves per SIMD, in bounds)
        constexpr int G9 = NCH >= 9 ? 9 : NCH;
        s4 cur[G9], nxt[G9];
#pragma unroll
        for (int m = 0; m < G9; ++m) cur[m] = tap(m);
#pragma unroll
        for (int g0 = 0; g0 < NCH; g0 += G9) {
            __builtin_amdgcn_sched_barrier(0);
            if (g0 + G9 < NCH) {
#pragma unroll
                for (int m = 0; m < G9; ++m) nxt[m] = g0 + G9 + m < NCH ? tap(g0 + G9 + m) : s4{0, 0, 0, 0};
            }
#pragma unroll
            for (int m = 0; m < G9; ++m)
                if (g0 + m < NCH) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(cur[m], wsh[g0 + m][lane], acc, 0, 0, 0);
#pragma unroll
            for (int m = 0; m < G9; ++m) cur[m] = nxt[m];
        }
        const int co = lane % 16;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t vo = tile * 16 + 4 * g + j;
            if (vo >= L.V) continue;
            float val = acc[j];
            if (MODE == 0) {
                val += bias[co];
                static_cast<uint16_t*>(out)[vo * 16 + co] = f2bf(val > 0.f ? val : 0.f);
            } else if (MODE == 1) {
                if (co == 0) static_cast<float*>(out)[vo] = val + bias[0];
            } else {
                const bool on = bf2f(mask[vo * 16 + co]) > 0.f;
                static_cast<uint16_t*>(out)[vo * 16 + co] = f2bf(on ? val : 0.f);
            }
        }
    }
}

// ---------------------------------------------------------------- weight gradients
// partial[w][m*256 + co*16 + n] = sum over this wavefront's lattice points of
// dZ[v][co] X[v + tap][ci], with (tap, ci) = (m, n) for CIN = 16 and
// (4m + n/4, n%4) for CIN = 4; partial[w][NCH*256 + co] = sum dZ[v][co].
template <int CIN>
__global__ __launch_bounds__(kThreads) void k_wgrad(Lat L, const uint16_t* __restrict__ dZ,
                                                    const uint16_t* __restrict__ X, float* __restrict__ partial) {
    constexpr int NCH = CIN == 16 ? 27 : 7;
    constexpr int STRIDE = NCH * 256 + 16;
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int g = lane / 16, n = lane % 16;
    const int64_t wg = (int64_t)blockIdx.x * 4 + wave;
    const int64_t nw = (int64_t)gridDim.x * 4;
    const int64_t ntiles = (L.V + 15) / 16;
    f4 acc[NCH];
#pragma unroll
    for (int m = 0; m < NCH; ++m) acc[m] = f4{0.f, 0.f, 0.f, 0.f};
    float db = 0.f;
    for (int64_t tile = wg; tile < ntiles; tile += nw) {
        s4 a;
        int64_t vv[4];
        int xs[4], ys[4], zs[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t v = tile * 16 + 4 * g + j;
            vv[j] = v;
            const bool ok = v < L.V;
            const uint16_t d = ok ? dZ[v * 16 + n] : uint16_t(0);
            a[j] = static_cast<short>(d);
            db += bf2f(d);
            xs[j] = static_cast<int>(v % L.nx);
            ys[j] = static_cast<int>((v / L.nx) % L.ny);
            zs[j] = static_cast<int>(v / ((int64_t)L.nx * L.ny));
        }
#pragma unroll
        for (int m = 0; m < NCH; ++m) {
            const int t = CIN == 16 ? m : 4 * m + n / 4;
            const int ci = CIN == 16 ? n : n % 4;
            s4 b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint16_t xv = 0;
                if (vv[j] < L.V && t < 27) {
                    const int64_t nb = neighbour(L, xs[j], ys[j], zs[j], t);
                    if (nb >= 0) xv = X[nb * CIN + ci];
                }
                b[j] = static_cast<short>(xv);
            }
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[m], 0, 0, 0);
        }
    }
    float* P = partial + wg * STRIDE;
#pragma unroll
    for (int m = 0; m < NCH; ++m)
#pragma unroll
        for (int j = 0; j < 4; ++j) P[m * 256 + (4 * g + j) * 16 + n] = acc[m][j];
    db += __shfl_xor(db, 16);
    db += __shfl_xor(db, 32);
    if (lane < 16) P[NCH * 256 + lane] = db;
}

// grad (canonical [co][ci][27] + [co]) of one layer = sum over wavefronts of the partials
template <int CIN>
__global__ void k_wgrad_reduce(const float* __restrict__ partial, int64_t nw, int cin, int cout,
                               float* __restrict__ grad) {
    constexpr int NCH = CIN == 16 ? 27 : 7;
    constexpr int STRIDE = NCH * 256 + 16;
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= STRIDE) return;
    float s = 0.f;
    for (int64_t w = 0; w < nw; ++w) s += partial[w * STRIDE + p];
    if (p >= NCH * 256) {
        const int co = p - NCH * 256;
        if (co < cout) grad[cout * cin * 27 + co] = s;
        return;
    }
    const int m = p / 256, co = (p / 16) % 16, nn = p % 16;
    const int tap = CIN == 16 ? m : 4 * m + nn / 4;
    const int ci = CIN == 16 ? nn : nn % 4;
    if (co < cout && ci < cin && tap < 27) grad[(co * cin + ci) * 27 + tap] = s;
}

// BF16 weights for the MFMA B operand, [m][n = output channel][k]:
// forward (trans = 0): n = co, k = ci (CIN 16) or k = 4 tl + ci, tap = 4m + tl (CIN 4)
// backward data (trans = 1): the adjoint convolution, n = ci, k = co, tap mirrored
__global__ void k_pack(const float* __restrict__ w, int cin, int cout, int nch, int trans, uint16_t* __restrict__ Wp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nch * 256) return;
    const int m = i / 256, n = (i / 16) % 16, k = i % 16;
    float val = 0.f;
    if (!trans) {
        int tap, ci;
        if (nch == 27) {
            tap = m;
            ci = k;
        } else {
            tap = 4 * m + k / 4;
            ci = k % 4;
        }
        if (n < cout && ci < cin && tap < 27) val = w[(n * cin + ci) * 27 + tap];
    } else {
        // dX[v][ci] = sum_tap' sum_co dZ[v + tap'][co] w[co][ci][26 - tap']
        const int tap = m, co = k, ci = n;
        if (co < cout && ci < cin) val = w[(co * cin + ci) * 27 + (26 - tap)];
    }
    Wp[i] = f2bf(val);
}

// The discrete fluence can dip slightly below zero far from the sources (the P1
// mass matrix has positive off-diagonal entries), so logs of fluences are
// taken of max(phi, kPhiFloor); corrections are clamped to e^{+-kMaxCorr}.
constexpr double kPhiFloor = 1e-16;
constexpr float kMaxCorr = 8.f;

// network input for illumination k: [V][4] bf16 = (log mu/mu0, log kappa/kappa0, log phi_hom, 0)
__global__ void k_inputs(int64_t V, const double* __restrict__ kappa, const double* __restrict__ mu, double k0,
                         double m0, const double* __restrict__ phih, uint16_t* __restrict__ X) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    X[v * 4 + 0] = f2bf(static_cast<float>(log(mu[v] / m0)));
    X[v * 4 + 1] = f2bf(static_cast<float>(log(kappa[v] / k0)));
    X[v * 4 + 2] = f2bf(static_cast<float>(log(fmax(phih[v], kPhiFloor))));
    X[v * 4 + 3] = 0;
}

// raw input [3][V] f32 -> [V][4] bf16
__global__ void k_inputs_raw(int64_t V, const float* __restrict__ in, uint16_t* __restrict__ X) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    X[v * 4 + 0] = f2bf(in[v]);
    X[v * 4 + 1] = f2bf(in[V + v]);
    X[v * 4 + 2] = f2bf(in[2 * V + v]);
    X[v * 4 + 3] = 0;
}

// target = log phi - log phi_hom (f32)
__global__ void k_target(int64_t V, const double* __restrict__ phi, const double* __restrict__ phih,
                         float* __restrict__ t) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    const double d = log(fmax(phi[v], kPhiFloor)) - log(fmax(phih[v], kPhiFloor));
    t[v] = static_cast<float>(fmin(fmax(d, -(double)kMaxCorr), (double)kMaxCorr));
}

// phi0 = phi_hom exp(pred)
__global__ void k_fluence(int64_t V, const float* __restrict__ pred, const double* __restrict__ phih,
                          double* __restrict__ phi0) {
    int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (v >= V) return;
    float p = pred[v];
    if (!(p == p)) p = 0.f;   // a non-finite prediction falls back to phi_hom
    p = fminf(fmaxf(p, -kMaxCorr), kMaxCorr);
    phi0[v] = phih[v] * exp(static_cast<double>(p));
}

// mean squared error: per-block partial sums; dZ4[v][0] = 2 (pred - t) / V
__global__ __launch_bounds__(kThreads) void k_loss(int64_t V, const float* __restrict__ pred,
                                                   const float* __restrict__ t, uint16_t* __restrict__ dZ,
                                                   double* __restrict__ part) {
    __shared__ double sm[kThreads / 64];
    double acc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < V; v += (int64_t)gridDim.x * blockDim.x) {
        const float d = pred[v] - t[v];
        acc += static_cast<double>(d) * d;
        dZ[v * 16] = f2bf(2.f * d / static_cast<float>(V));
#pragma unroll
        for (int c = 1; c < 16; ++c) dZ[v * 16 + c] = 0;
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) s += sm[w];
        part[blockIdx.x] = s;
    }
}

__global__ void k_loss_final(const double* __restrict__ part, int nb, int64_t V, double* __restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[b];
    *out = s / static_cast<double>(V);
}

// Adam on the FP32 master parameters (Kingma and Ba's update with bias correction)
__global__ void k_adam(int n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float a = b1 * m1[i] + (1.f - b1) * gi;
    const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
    m1[i] = a;
    m2[i] = b;
    w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_zero_f(int n, float* p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

constexpr int kConvBlocks = 2048;   // 8192 wavefronts over 256 CUs

int nch_of(int layer) { return layer == 0 ? 7 : 27; }

}  // namespace

// ---------------------------------------------------------------- host side
struct GuessNet {
    Lat L{};
    float* params = nullptr;   // [kParams] FP32 master
    float* grads = nullptr;
    float* m1 = nullptr;
    float* m2 = nullptr;
    uint16_t* Wf[kLayers] = {};  // forward B operands
    uint16_t* Wb[kLayers] = {};  // backward-data B operands
    uint16_t* X0 = nullptr;      // [V][4]
    uint16_t* Y[3] = {};         // hidden activations [V][16]
    uint16_t* dA = nullptr;      // [V][16]
    uint16_t* dB = nullptr;      // [V][16]
    float* pred = nullptr;       // [V]
    float* target = nullptr;     // [V]
    float* partial = nullptr;    // [waves][27*256+16]
    double* lossp = nullptr;     // [blocks]
    double* lossv = nullptr;     // [1]
    int step = 0;
};

static qpat_status guess_pack(qpat_ctx* c) {
    GuessNet* G = c->guess;
    for (int l = 0; l < kLayers; ++l) {
        const float* w = G->params + param_offset(l);
        const int nch = nch_of(l);
        hipLaunchKernelGGL(k_pack, dim3((nch * 256 + 255) / 256), dim3(256), 0, c->stream, w, kCin[l], kCout[l], nch, 0,
                           G->Wf[l]);
        if (l > 0)
            hipLaunchKernelGGL(k_pack, dim3(27), dim3(256), 0, c->stream, w, kCin[l], kCout[l], 27, 1, G->Wb[l]);
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// forward pass; the last layer writes its single output channel, FP32 [V]
static qpat_status guess_forward(qpat_ctx* c, float* out) {
    GuessNet* G = c->guess;
    const dim3 g(kConvBlocks), b(kThreads);
    const float* bias[kLayers];
    for (int l = 0; l < kLayers; ++l) bias[l] = G->params + param_offset(l) + kCout[l] * kCin[l] * 27;
    hipLaunchKernelGGL((k_conv<4, 0>), g, b, 0, c->stream, G->L, G->X0, G->Wf[0], bias[0], nullptr, (void*)G->Y[0]);
    hipLaunchKernelGGL((k_conv<16, 0>), g, b, 0, c->stream, G->L, G->Y[0], G->Wf[1], bias[1], nullptr, (void*)G->Y[1]);
    hipLaunchKernelGGL((k_conv<16, 0>), g, b, 0, c->stream, G->L, G->Y[1], G->Wf[2], bias[2], nullptr, (void*)G->Y[2]);
    hipLaunchKernelGGL((k_conv<16, 1>), g, b, 0, c->stream, G->L, G->Y[2], G->Wf[3], bias[3], nullptr, (void*)out);
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

// loss and gradients of the current sample (input in X0, target in G->target)
static qpat_status guess_backward(qpat_ctx* c) {
    GuessNet* G = c->guess;
    const int64_t V = G->L.V;
    const dim3 g(kConvBlocks), b(kThreads);
    const int lb = grid_for(V, kThreads, 1024);
    QPAT_TRY(guess_forward(c, G->pred));
    hipLaunchKernelGGL(k_loss, dim3(lb), b, 0, c->stream, V, G->pred, G->target, G->dA, G->lossp);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, c->stream, G->lossp, lb, V, G->lossv);
    const int64_t nw = (int64_t)kConvBlocks * 4;
    // dZ of layer l in cur; its input activation is Y[l-1] (X0 for l = 0)
    uint16_t* cur = G->dA;
    uint16_t* nxt = G->dB;
    for (int l = kLayers - 1; l >= 0; --l) {
        const uint16_t* Xin = l == 0 ? G->X0 : G->Y[l - 1];
        float* grad = G->grads + param_offset(l);
        if (l == 0) {
            hipLaunchKernelGGL(k_wgrad<4>, g, b, 0, c->stream, G->L, cur, Xin, G->partial);
            hipLaunchKernelGGL(k_wgrad_reduce<4>, dim3((7 * 256 + 16 + 255) / 256), dim3(256), 0, c->stream,
                               G->partial, nw, kCin[l], kCout[l], grad);
        } else {
            hipLaunchKernelGGL(k_wgrad<16>, g, b, 0, c->stream, G->L, cur, Xin, G->partial);
            hipLaunchKernelGGL(k_wgrad_reduce<16>, dim3((27 * 256 + 16 + 255) / 256), dim3(256), 0, c->stream,
                               G->partial, nw, kCin[l], kCout[l], grad);
            // dZ of layer l-1 = (adjoint convolution of dZ_l) masked by ReLU(Y[l-1]) > 0
            hipLaunchKernelGGL((k_conv<16, 2>), g, b, 0, c->stream, G->L, cur, G->Wb[l], nullptr, G->Y[l - 1],
                               (void*)nxt);
            uint16_t* t = cur;
            cur = nxt;
            nxt = t;
        }
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

qpat_status guess_setup(qpat_ctx* c, int nx, int ny, int nz) {
    if ((int64_t)nx * ny * nz != c->N) return fail(c, QPAT_ERR_ARG, "guess_setup: nx*ny*nz must equal N");
    if (c->N * 16 * 2 >= (int64_t(1) << 31))   // the convolutions' 32-bit buffer offsets
        return fail(c, QPAT_ERR_ARG, "guess_setup: lattice too large for the network (N = %lld)", (long long)c->N);
    if (!c->guess) c->guess = new GuessNet();
    GuessNet* G = c->guess;
    if (G->L.V == c->N && G->params) return QPAT_OK;
    G->L = Lat{nx, ny, nz, c->N};
    const int64_t V = c->N;
    QPAT_TRY(dalloc(c, &G->params, kParams));
    QPAT_TRY(dalloc(c, &G->grads, kParams));
    QPAT_TRY(dalloc(c, &G->m1, kParams));
    QPAT_TRY(dalloc(c, &G->m2, kParams));
    for (int l = 0; l < kLayers; ++l) {
        QPAT_TRY(dalloc(c, &G->Wf[l], (size_t)nch_of(l) * 256));
        QPAT_TRY(dalloc(c, &G->Wb[l], (size_t)27 * 256));
    }
    QPAT_TRY(dalloc(c, &G->X0, V * 4));
    for (int l = 0; l < 3; ++l) QPAT_TRY(dalloc(c, &G->Y[l], V * 16));
    QPAT_TRY(dalloc(c, &G->dA, V * 16));
    QPAT_TRY(dalloc(c, &G->dB, V * 16));
    QPAT_TRY(dalloc(c, &G->pred, V));
    QPAT_TRY(dalloc(c, &G->target, V));
    QPAT_TRY(dalloc(c, &G->partial, (size_t)kConvBlocks * 4 * (27 * 256 + 16)));
    QPAT_TRY(dalloc(c, &G->lossp, 1024));
    QPAT_TRY(dalloc(c, &G->lossv, 1));
    hipLaunchKernelGGL(k_zero_f, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, kParams, G->params);
    QPAT_TRY(guess_pack(c));
    return QPAT_OK;
}

qpat_status guess_set_params(qpat_ctx* c, const float* p) {
    GuessNet* G = c->guess;
    QPAT_HIP(c, hipMemcpyAsync(G->params, p, sizeof(float) * kParams, hipMemcpyDeviceToDevice, c->stream));
    hipLaunchKernelGGL(k_zero_f, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, kParams, G->m1);
    hipLaunchKernelGGL(k_zero_f, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, kParams, G->m2);
    G->step = 0;
    return guess_pack(c);
}

qpat_status guess_get_params(qpat_ctx* c, float* p) {
    QPAT_HIP(c, hipMemcpyAsync(p, c->guess->params, sizeof(float) * kParams, hipMemcpyDeviceToDevice, c->stream));
    return QPAT_OK;
}

qpat_status guess_eval_raw(qpat_ctx* c, const float* in, float* out) {
    GuessNet* G = c->guess;
    hipLaunchKernelGGL(k_inputs_raw, dim3(grid_for(G->L.V, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream,
                       G->L.V, in, G->X0);
    return guess_forward(c, out);
}

qpat_status guess_grad_raw(qpat_ctx* c, const float* in, const float* target, float* grad, double* loss) {
    GuessNet* G = c->guess;
    hipLaunchKernelGGL(k_inputs_raw, dim3(grid_for(G->L.V, kThreads, 1 << 30)), dim3(kThreads), 0, c->stream,
                       G->L.V, in, G->X0);
    QPAT_HIP(c, hipMemcpyAsync(G->target, target, sizeof(float) * G->L.V, hipMemcpyDeviceToDevice, c->stream));
    QPAT_TRY(guess_backward(c));
    if (grad) QPAT_HIP(c, hipMemcpyAsync(grad, G->grads, sizeof(float) * kParams, hipMemcpyDeviceToDevice, c->stream));
    QPAT_HIP(c, hipMemcpyAsync(c->red_host, G->lossv, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    QPAT_HIP(c, hipStreamSynchronize(c->stream));
    if (loss) *loss = c->red_host[0];
    return QPAT_OK;
}

static qpat_status adam_step(qpat_ctx* c, float lr) {
    GuessNet* G = c->guess;
    G->step += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)G->step), c2 = 1.f - std::pow(b2, (float)G->step);
    hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, c->stream, kParams, G->params, G->grads,
                       G->m1, G->m2, lr, b1, b2, 1e-8f, c1, c2);
    return guess_pack(c);
}

// one Adam step on the sample of illumination k: input from (kappa, mu, phi_hom_k), target log(phi_k / phi_hom_k)
qpat_status guess_train(qpat_ctx* c, const double* kappa, const double* mu, double k0, double m0,
                        const double* phih, const double* phi, float lr, double* loss) {
    GuessNet* G = c->guess;
    const dim3 gg(grid_for(G->L.V, kThreads, 1 << 30)), b(kThreads);
    hipLaunchKernelGGL(k_inputs, gg, b, 0, c->stream, G->L.V, kappa, mu, k0, m0, phih, G->X0);
    hipLaunchKernelGGL(k_target, gg, b, 0, c->stream, G->L.V, phi, phih, G->target);
    QPAT_TRY(guess_backward(c));
    QPAT_TRY(adam_step(c, lr));
    if (loss) {
        QPAT_HIP(c, hipMemcpyAsync(c->red_host, G->lossv, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        QPAT_HIP(c, hipStreamSynchronize(c->stream));
        *loss = c->red_host[0];
    }
    return QPAT_OK;
}

qpat_status guess_train_raw(qpat_ctx* c, const float* in, const float* target, float lr, double* loss) {
    QPAT_TRY(guess_grad_raw(c, in, target, nullptr, loss));
    return adam_step(c, lr);
}

// phi0_k = phi_hom_k exp(net(log mu/mu0, log kappa/kappa0, log phi_hom_k)) for every illumination
qpat_status guess_fluence(qpat_ctx* c, const double* kappa, const double* mu, double k0, double m0,
                          const double* phih, double* phi0) {
    GuessNet* G = c->guess;
    const int64_t V = G->L.V;
    const dim3 gg(grid_for(V, kThreads, 1 << 30)), b(kThreads);
    for (int k = 0; k < c->n_ill; ++k) {
        hipLaunchKernelGGL(k_inputs, gg, b, 0, c->stream, V, kappa, mu, k0, m0, phih + k * V, G->X0);
        QPAT_TRY(guess_forward(c, G->pred));
        hipLaunchKernelGGL(k_fluence, gg, b, 0, c->stream, V, G->pred, phih + k * V, phi0 + k * V);
    }
    QPAT_HIP(c, hipGetLastError());
    return QPAT_OK;
}

void guess_destroy(qpat_ctx* c) {
    delete c->guess;
    c->guess = nullptr;
}

}  // namespace qpat
