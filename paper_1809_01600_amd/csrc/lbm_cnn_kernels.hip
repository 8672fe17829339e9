// HIP kernels (gfx950) of the learned warm start: 3x3 convolution forward / backward, masked MSE,
// Adam, and the feature / assembly kernels that connect the network to the LBM solver.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <mutex>
#include <type_traits>

#include "lbm_cnn.h"

namespace lbmcnn {

constexpr int TS = 16;         // output tile edge (pixels); workgroup = TS x TS lanes
constexpr int HALO = TS + 2;   // input tile edge
constexpr int CCH = 8;         // input channels staged per pass
constexpr int MAXC = 32;       // largest channel count
constexpr int WG_PARTIALS = 1024;  // upper bound on backward-weight workgroups

__device__ inline float bf16_to_f32(uint16_t h)
{
    return __uint_as_float(((uint32_t)h) << 16);
}

// round to nearest even
__device__ inline uint16_t f32_to_bf16(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <class T> __device__ inline float ld(const T* p, long long i);
template <> __device__ inline float ld<float>(const float* p, long long i) { return p[i]; }
template <> __device__ inline float ld<uint16_t>(const uint16_t* p, long long i) { return bf16_to_f32(p[i]); }
template <class T> __device__ inline void st(T* p, long long i, float v);
template <> __device__ inline void st<float>(float* p, long long i, float v) { p[i] = v; }
template <> __device__ inline void st<uint16_t>(uint16_t* p, long long i, float v) { p[i] = f32_to_bf16(v); }

// out[b][co][y][x] = act(bias[co] + sum_ci sum_k w[co][ci][k] * in'[b][ci][y+ky-1][x+kx-1]),
// in' = in * (gate > 0) when gate is given.  One workgroup = one 16x16 tile of one image, all
// output channels per lane (COUT accumulators); weights in LDS (broadcast reads).
template <class T, class WT, int COUT>
__global__ __launch_bounds__(TS * TS) void k_conv_fwd(const T* __restrict__ in,
                                                      const float* __restrict__ gate, int Cin,
                                                      int H, int W, const WT* __restrict__ w,
                                                      const float* __restrict__ bias, int relu,
                                                      T* __restrict__ out)
{
    __shared__ float sW[COUT * MAXC * 9];
    __shared__ float sIn[CCH][HALO][HALO];
    const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
    const int x = blockIdx.x * TS + tx, y = blockIdx.y * TS + ty;
    const int b = blockIdx.z;
    const long long plane = (long long)H * W;
    for (int i = threadIdx.x; i < COUT * Cin * 9; i += TS * TS) sW[i] = ld<WT>(w, i);
    float acc[COUT];
#pragma unroll
    for (int co = 0; co < COUT; ++co) acc[co] = bias ? bias[co] : 0.f;
    for (int c0 = 0; c0 < Cin; c0 += CCH) {
        __syncthreads();
        for (int i = threadIdx.x; i < CCH * HALO * HALO; i += TS * TS) {
            const int c = i / (HALO * HALO), r = i % (HALO * HALO);
            const int gy = blockIdx.y * TS + r / HALO - 1, gx = blockIdx.x * TS + r % HALO - 1;
            float v = 0.f;
            if (c0 + c < Cin && gy >= 0 && gy < H && gx >= 0 && gx < W) {
                const long long gi = ((long long)b * Cin + c0 + c) * plane + (long long)gy * W + gx;
                v = ld<T>(in, gi);
                if (gate && !(gate[gi] > 0.f)) v = 0.f;
            }
            sIn[c][r / HALO][r % HALO] = v;
        }
        __syncthreads();
        const int cn = min(CCH, Cin - c0);
        for (int c = 0; c < cn; ++c)
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const float v = sIn[c][ty + k / 3][tx + k % 3];
                const float* wk = &sW[(c0 + c) * 9 + k];
#pragma unroll
                for (int co = 0; co < COUT; ++co) acc[co] += wk[co * Cin * 9] * v;
            }
    }
    if (x < W && y < H) {
#pragma unroll
        for (int co = 0; co < COUT; ++co) {
            float o = acc[co];
            if (relu) o = o > 0.f ? o : 0.f;
            st<T>(out, ((long long)b * COUT + co) * plane + (long long)y * W + x, o);
        }
    }
}

// w^T[ci][co][8 - k] = w[co][ci][k]
__global__ void k_transpose_flip(const float* __restrict__ w, int Cout, int Cin, float* __restrict__ wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Cout * Cin * 9) return;
    const int k = i % 9, ci = (i / 9) % Cin, co = i / (9 * Cin);
    wt[(ci * Cout + co) * 9 + (8 - k)] = w[i];
}

// Per-workgroup partial sums of grad_w[co][ci][k] and grad_b[co] over a run of 16x16 tiles.
// Lane t owns up to four (co, ci) pairs (all nine taps each); lanes < Cout also sum the bias.
__global__ __launch_bounds__(TS * TS) void k_conv_bwd_w(const float* __restrict__ in,
                                                        const float* __restrict__ go,
                                                        const float* __restrict__ act, int B,
                                                        int Cin, int Cout, int H, int W,
                                                        int tiles_per_wg, float* __restrict__ partial)
{
    __shared__ float sGo[MAXC][TS * TS];
    __shared__ float sIn[MAXC][HALO * HALO];
    const int tilesx = (W + TS - 1) / TS, tilesy = (H + TS - 1) / TS;
    const int ntiles = B * tilesx * tilesy;
    const int npairs = Cout * Cin;
    const long long plane = (long long)H * W;
    float acc[4][9];
    float accb = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[r][k] = 0.f;
    const int t0 = blockIdx.x * tiles_per_wg;
    for (int tt = t0; tt < min(t0 + tiles_per_wg, ntiles); ++tt) {
        const int b = tt / (tilesx * tilesy);
        const int rr = tt % (tilesx * tilesy);
        const int bx = rr % tilesx, by = rr / tilesx;
        __syncthreads();
        for (int i = threadIdx.x; i < Cout * TS * TS; i += TS * TS) {
            const int co = i / (TS * TS), p = i % (TS * TS);
            const int gy = by * TS + p / TS, gx = bx * TS + p % TS;
            float v = 0.f;
            if (gy < H && gx < W) {
                const long long gi = ((long long)b * Cout + co) * plane + (long long)gy * W + gx;
                v = go[gi];
                if (act && !(act[gi] > 0.f)) v = 0.f;
            }
            sGo[co][p] = v;
        }
        for (int i = threadIdx.x; i < Cin * HALO * HALO; i += TS * TS) {
            const int c = i / (HALO * HALO), r = i % (HALO * HALO);
            const int gy = by * TS + r / HALO - 1, gx = bx * TS + r % HALO - 1;
            float v = 0.f;
            if (gy >= 0 && gy < H && gx >= 0 && gx < W)
                v = in[((long long)b * Cin + c) * plane + (long long)gy * W + gx];
            sIn[c][r] = v;
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pr = threadIdx.x + r * TS * TS;
            if (pr >= npairs) break;
            const int co = pr / Cin, ci = pr % Cin;
            for (int p = 0; p < TS * TS; ++p) {
                const float g = sGo[co][p];
                const int py = p / TS, px = p % TS;
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[r][k] += g * sIn[ci][(py + k / 3) * HALO + px + k % 3];
            }
        }
        if (threadIdx.x < (unsigned)Cout)
            for (int p = 0; p < TS * TS; ++p) accb += sGo[threadIdx.x][p];
    }
    float* out = partial + (long long)blockIdx.x * (npairs * 9 + Cout);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int pr = threadIdx.x + r * TS * TS;
        if (pr >= npairs) break;
#pragma unroll
        for (int k = 0; k < 9; ++k) out[pr * 9 + k] = acc[r][k];
    }
    if (threadIdx.x < (unsigned)Cout) out[npairs * 9 + threadIdx.x] = accb;
}

// fixed-order sum of the per-workgroup partials
__global__ void k_sum_partials(const float* __restrict__ partial, int nwg, int nw, int nb,
                               float* __restrict__ gw, float* __restrict__ gb)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw + nb) return;
    float s = 0.f;
    for (int g = 0; g < nwg; ++g) s += partial[(long long)g * (nw + nb) + i];
    if (i < nw) gw[i] = s;
    else gb[i - nw] = s;
}

// pass 1: unnormalized gradient 2 m (p - t) and per-workgroup sums of m (p - t)^2 and m
__global__ __launch_bounds__(256) void k_masked_mse(const float* __restrict__ pred,
                                                    const float* __restrict__ tgt,
                                                    const float* __restrict__ fluid, int B, int C,
                                                    int H, int W, float* __restrict__ grad,
                                                    double* __restrict__ partial)
{
    __shared__ double red[2][4];
    const long long plane = (long long)H * W;
    const long long n = (long long)B * C * plane;
    double se = 0.0, cnt = 0.0;
    for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        const long long p = i % plane, b = i / (C * plane);
        const float m = fluid[b * plane + p];
        const float d = pred[i] - tgt[i];
        se += (double)(m * d * d);
        cnt += (double)m;
        grad[i] = 2.f * m * d;
    }
    for (int off = 32; off > 0; off >>= 1) {
        se += __shfl_down(se, off, 64);
        cnt += __shfl_down(cnt, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = se;
        red[1][threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        partial[2 * blockIdx.x + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// pass 2 (one lane): loss = sum / count in fixed order; 1 / count for pass 3
__global__ void k_mse_finalize(const double* __restrict__ partial, int nwg, double* __restrict__ loss,
                               double* __restrict__ inv_count)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double se = 0.0, cnt = 0.0;
    for (int g = 0; g < nwg; ++g) {
        se += partial[2 * g];
        cnt += partial[2 * g + 1];
    }
    loss[0] = cnt > 0 ? se / cnt : 0.0;
    inv_count[0] = cnt > 0 ? 1.0 / cnt : 0.0;
}

// pass 3: grad /= count
__global__ void k_scale(float* __restrict__ g, long long n, const double* __restrict__ s)
{
    const float f = (float)s[0];
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        g[i] *= f;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps,
                       float c1, float c2)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

__global__ void k_to_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = f32_to_bf16(in[i]);
}

__global__ void k_from_bf16(const uint16_t* __restrict__ in, float* __restrict__ out, long long n)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[i] = bf16_to_f32(in[i]);
}

// Feature rows [y0, y0 + FEAT_ROWS) of instance blockIdx.y.  Every workgroup first rebuilds the
// per-column fluid fraction phi(x) and the porosity-weighted profile in LDS (a column scan per
// species), then writes its rows of the eight channels; the first row block also writes the
// profile itself (the baseline the prediction corrects).
constexpr int FEAT_ROWS = 16;
constexpr int FEAT_MAX_W = 2048;  // LDS: 4 W + 16 W bytes
constexpr float DEPLETION_SCALE = 0.01f;

__global__ void __launch_bounds__(256) k_features(const uint8_t* __restrict__ solid,
                                                  const double* __restrict__ X_in,
                                                  const double* __restrict__ j,
                                                  const double* __restrict__ prof, int H, int W,
                                                  float* __restrict__ feat,
                                                  double* __restrict__ base)
{
    extern __shared__ int lds[];
    int* cnt = lds;                                                   // [W] fluid per column
    double* pp = reinterpret_cast<double*>(lds + 2 * ((W + 1) / 2));  // [2][W], 8-byte aligned
    const int b = blockIdx.y;
    const long long plane = (long long)H * W;
    const uint8_t* sb = solid + b * plane;
    for (int x = threadIdx.x; x < W; x += blockDim.x) {
        int c = 0;
        for (int y = 0; y < H; ++y) c += sb[(long long)y * W + x] ? 0 : 1;
        cnt[x] = c > 0 ? c : 1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int sp = threadIdx.x;
        const double* pr = prof + (long long)(b * 2 + sp) * W;
        double prev = X_in[3 * b + sp], acc = prev;
        for (int x = 0; x < W; ++x) {
            const double v = pr[x];
            acc += (v - prev) * (double)H / (double)cnt[x];
            prev = v;
            pp[sp * W + x] = acc;
        }
    }
    __syncthreads();
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 2 * W; i += blockDim.x) base[(long long)b * 2 * W + i] = pp[i];
    const int y0 = blockIdx.x * FEAT_ROWS;
    const int rows = min(FEAT_ROWS, H - y0);
    float* fb = feat + b * 8 * plane;
    const double x1 = X_in[3 * b], x2 = X_in[3 * b + 1];
    const float jj = (float)(0.5 * j[b]);
    const float rw = W > 1 ? 1.f / (float)(W - 1) : 0.f;
    for (int i = threadIdx.x; i < rows * W; i += blockDim.x) {
        const int x = i % W;
        const long long p = (long long)(y0 + i / W) * W + x;
        fb[p] = sb[p] ? 0.f : 1.f;
        fb[plane + p] = (float)x1;
        fb[2 * plane + p] = (float)x2;
        fb[3 * plane + p] = jj;
        fb[4 * plane + p] = (float)x * rw;
        fb[5 * plane + p] = (float)(pp[x] - x1) / DEPLETION_SCALE;
        fb[6 * plane + p] = (float)(pp[W + x] - x2) / DEPLETION_SCALE;
        fb[7 * plane + p] = (float)cnt[x] / (float)H;
    }
}

__global__ void k_assemble(const float* __restrict__ pred, const double* __restrict__ prof, int B,
                           int H, int W, float scale, double x_min, double* __restrict__ X)
{
    const long long plane = (long long)H * W;
    const long long n = (long long)B * plane;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long b = i / plane, p = i % plane;
        const int x = (int)(p % W);
        double x1 = prof[(b * 2) * W + x] + (double)scale * pred[(b * 2) * plane + p];
        double x2 = prof[(b * 2 + 1) * W + x] + (double)scale * pred[(b * 2 + 1) * plane + p];
        x1 = x1 > x_min ? x1 : x_min;
        x2 = x2 > x_min ? x2 : x_min;
        double x3 = 1.0 - x1 - x2;
        if (x3 < x_min) {  // take the excess from the parts of X_1, X_2 above x_min
            const double s = (1.0 - 3.0 * x_min) / (x1 + x2 - 2.0 * x_min);
            x1 = x_min + (x1 - x_min) * s;
            x2 = x_min + (x2 - x_min) * s;
            x3 = 1.0 - x1 - x2;
        }
        X[(b * 3) * plane + p] = x1;
        X[(b * 3 + 1) * plane + p] = x2;
        X[(b * 3 + 2) * plane + p] = x3;
    }
}

inline int grid_for(long long n, int bs = 256, int cap = 8192)
{
    long long g = (n + bs - 1) / bs;
    return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

inline int status(hipError_t e) { return e == hipSuccess ? 0 : -4; }

// BF16 convolution on the matrix cores: 32 output channels from CIN = 8 or 32 input channels, as
// the implicit GEMM out[pixel][co] = sum_kk A[pixel][kk] W[kk][co] with kk = tap * CIN + ci (taps
// 0..8 row-major over the 3x3 window), in K chunks of 32 by v_mfma_f32_16x16x32_bf16 (FP32
// accumulation).  One workgroup = one 16x16 pixel tile of one image, four waves; wave v owns tile
// rows 4v..4v+3 (one 16-pixel M block each) and both 16-channel N blocks.  LDS holds the 18x18
// input tile pixel-major (the CIN channels of a pixel together) and the weights as [tap][co][ci],
// so each lane's eight K values of an operand are one 16-byte read: A lane l takes pixel l % 16
// of its row and kk = 32 m + 8 (l / 16) .. + 7, B lane l takes channel l % 16 of its block and the
// same kk; D lane l holds rows (pixels) 4 (l / 16) + j, j = 0..3, of channel l % 16.  A K chunk
// past tap 8 (CIN = 8: 72 = 9 x 8 kk padded to 96) reads zeros.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int CIN>
__global__ __launch_bounds__(256) void k_conv_fwd_mfma(const uint16_t* __restrict__ in, int H, int W,
                                                       const uint16_t* __restrict__ w,
                                                       const float* __restrict__ bias, int relu,
                                                       uint16_t* __restrict__ out)
{
    constexpr int COUT = 32, KCH = (9 * CIN + 31) / 32;  // K chunks of 32
    __shared__ __align__(16) uint16_t sIn[HALO * HALO * CIN];
    __shared__ __align__(16) uint16_t sW[(KCH * 32 / CIN) * COUT * CIN];  // taps padded to the chunks
    const int b = blockIdx.z;
    const long long plane = (long long)H * W;
    const int tx0 = blockIdx.x * TS, ty0 = blockIdx.y * TS;
    // stage: weights w[co][ci][tap] -> sW[tap][co][ci] (padding taps zero), inputs NCHW -> [pix][ci]
    for (int i = threadIdx.x; i < (KCH * 32 / CIN) * COUT * CIN; i += 256) {
        const int ci = i % CIN, co = (i / CIN) % COUT, tap = i / (CIN * COUT);
        sW[i] = tap < 9 ? w[(co * CIN + ci) * 9 + tap] : (uint16_t)0;
    }
    for (int i = threadIdx.x; i < CIN * HALO * HALO; i += 256) {
        const int c = i / (HALO * HALO), r = i % (HALO * HALO);
        const int gy = ty0 + r / HALO - 1, gx = tx0 + r % HALO - 1;
        uint16_t v = 0;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W)
            v = in[((long long)b * CIN + c) * plane + (long long)gy * W + gx];
        sIn[r * CIN + c] = v;
    }
    __syncthreads();
    const int l = threadIdx.x & 63, v = threadIdx.x >> 6;
    const int lr = l & 15, lg = l >> 4;
    f32x4 acc[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 2; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KCH; ++kc) {
        const int kk = kc * 32 + lg * 8;  // this lane group's first K index
        const int tap = kk / CIN, ci0 = kk % CIN;
        const int ky = tap < 9 ? tap / 3 : 0, kx = tap < 9 ? tap % 3 : 0;
        bf16x8 bw[2];
#pragma unroll
        for (int n = 0; n < 2; ++n)
            bw[n] = *reinterpret_cast<const bf16x8*>(&sW[(tap * COUT + n * 16 + lr) * CIN + ci0]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int py = 4 * v + m;  // tile row of this M block; pixel x = lr
            bf16x8 a = *reinterpret_cast<const bf16x8*>(&sIn[((py + ky) * HALO + lr + kx) * CIN + ci0]);
            if (tap >= 9) a = bf16x8{};  // padded K: zero operand
#pragma unroll
            for (int n = 0; n < 2; ++n) acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw[n], acc[m][n], 0, 0, 0);
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const int y = ty0 + 4 * v + m;
        if (y >= H) continue;
#pragma unroll
        for (int n = 0; n < 2; ++n) {
            const int co = n * 16 + lr;
            const float bb = bias ? bias[co] : 0.f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int x = tx0 + 4 * lg + j;
                float o = acc[m][n][j] + bb;
                if (relu) o = o > 0.f ? o : 0.f;
                if (x < W) out[((long long)b * COUT + co) * plane + (long long)y * W + x] = f32_to_bf16(o);
            }
        }
    }
}

template <class T, class WT>
int conv_forward(const T* in, const float* gate, int B, int Cin, int H, int W, const WT* w,
                 const float* b, int Cout, int relu, T* out, hipStream_t st)
{
    if (!in || !w || !out || B <= 0 || H <= 0 || W <= 0 || Cin <= 0 || Cin > MAXC) return -1;
    const dim3 grid((W + TS - 1) / TS, (H + TS - 1) / TS, B);
    if constexpr (std::is_same<T, uint16_t>::value && std::is_same<WT, uint16_t>::value) {
        // BF16 inference: the 32-channel layers on the matrix cores
        if (Cout == 32 && !gate && (Cin == 8 || Cin == 32)) {
            if (Cin == 8) hipLaunchKernelGGL((k_conv_fwd_mfma<8>), grid, dim3(256), 0, st, in, H, W, w, b, relu, out);
            else hipLaunchKernelGGL((k_conv_fwd_mfma<32>), grid, dim3(256), 0, st, in, H, W, w, b, relu, out);
            return status(hipGetLastError());
        }
    }
    switch (Cout) {
    case 32: hipLaunchKernelGGL((k_conv_fwd<T, WT, 32>), grid, dim3(TS * TS), 0, st, in, gate, Cin, H, W, w, b, relu, out); break;
    case 8: hipLaunchKernelGGL((k_conv_fwd<T, WT, 8>), grid, dim3(TS * TS), 0, st, in, gate, Cin, H, W, w, b, relu, out); break;
    case 2: hipLaunchKernelGGL((k_conv_fwd<T, WT, 2>), grid, dim3(TS * TS), 0, st, in, gate, Cin, H, W, w, b, relu, out); break;
    default: return -1;
    }
    return status(hipGetLastError());
}

}  // namespace lbmcnn

using namespace lbmcnn;

extern "C" {

int lbm_cnn_conv_forward(const float* in, const float* gate, int B, int C_in, int H, int W,
                         const float* w, const float* b, int C_out, int relu, float* out,
                         void* stream)
{
    return conv_forward<float, float>(in, gate, B, C_in, H, W, w, b, C_out, relu, out,
                                      (hipStream_t)stream);
}

int lbm_cnn_conv_forward_bf16(const uint16_t* in, int B, int C_in, int H, int W,
                              const uint16_t* w, const float* b, int C_out, int relu,
                              uint16_t* out, void* stream)
{
    return conv_forward<uint16_t, uint16_t>(in, nullptr, B, C_in, H, W, w, b, C_out, relu, out,
                                            (hipStream_t)stream);
}

int lbm_cnn_conv_backward_data(const float* grad_out, const float* act, int B, int C_out, int H,
                               int W, const float* w, int C_in, float* grad_in, float* wt_scratch,
                               void* stream)
{
    if (!grad_out || !w || !grad_in || !wt_scratch || C_out <= 0 || C_out > MAXC) return -1;
    hipStream_t st = (hipStream_t)stream;
    const int n = C_out * C_in * 9;
    hipLaunchKernelGGL(k_transpose_flip, dim3((n + 255) / 256), dim3(256), 0, st, w, C_out, C_in, wt_scratch);
    const int e = status(hipGetLastError());
    if (e) return e;
    return conv_forward<float, float>(grad_out, act, B, C_out, H, W, wt_scratch, nullptr, C_in, 0,
                                      grad_in, st);
}

static int bwd_w_groups(int B, int H, int W, int* tiles_per)
{
    const long long ntiles = (long long)B * ((W + TS - 1) / TS) * ((H + TS - 1) / TS);
    const long long tp = (ntiles + WG_PARTIALS - 1) / WG_PARTIALS;
    *tiles_per = (int)(tp < 1 ? 1 : tp);
    return (int)((ntiles + *tiles_per - 1) / *tiles_per);
}

size_t lbm_cnn_backward_weight_scratch(int B, int C_in, int C_out, int H, int W)
{
    int tp;
    const int nwg = bwd_w_groups(B, H, W, &tp);
    return (size_t)nwg * (size_t)(C_out * C_in * 9 + C_out);
}

int lbm_cnn_conv_backward_weight(const float* in, const float* grad_out, const float* act, int B,
                                 int C_in, int C_out, int H, int W, float* grad_w, float* grad_b,
                                 float* partial, void* stream)
{
    if (!in || !grad_out || !grad_w || !grad_b || !partial) return -1;
    if (C_in <= 0 || C_in > MAXC || C_out <= 0 || C_out > MAXC || C_in * C_out > 4 * TS * TS)
        return -1;
    hipStream_t st = (hipStream_t)stream;
    int tp;
    const int nwg = bwd_w_groups(B, H, W, &tp);
    hipLaunchKernelGGL(k_conv_bwd_w, dim3(nwg), dim3(TS * TS), 0, st, in, grad_out, act, B, C_in,
                       C_out, H, W, tp, partial);
    int e = status(hipGetLastError());
    if (e) return e;
    const int nw = C_out * C_in * 9;
    hipLaunchKernelGGL(k_sum_partials, dim3((nw + C_out + 255) / 256), dim3(256), 0, st, partial,
                       nwg, nw, C_out, grad_w, grad_b);
    return status(hipGetLastError());
}

int lbm_cnn_masked_mse(const float* pred, const float* target, const float* fluid, int B, int C,
                       int H, int W, float* grad, double* loss_out, double* partial,
                       void* stream)
{
    if (!pred || !target || !fluid || !grad || !loss_out || !partial) return -1;
    hipStream_t st = (hipStream_t)stream;
    const long long n = (long long)B * C * H * W;
    const int g = grid_for(n, 256, 1024);
    hipLaunchKernelGGL(k_masked_mse, dim3(g), dim3(256), 0, st, pred, target, fluid, B, C, H, W,
                       grad, partial);
    int e = status(hipGetLastError());
    if (e) return e;
    hipLaunchKernelGGL(k_mse_finalize, dim3(1), dim3(64), 0, st, partial, g, loss_out, partial + 2 * 1024);
    e = status(hipGetLastError());
    if (e) return e;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, st, grad, n, partial + 2 * 1024);
    return status(hipGetLastError());
}

// Scratch of lbm_cnn_masked_mse_noalloc: the same 2 * 1024 + 1 float64 that lbm_cnn_masked_mse
// takes as `partial` (two sums per pass-1 workgroup, at most 1024 workgroups, then 1 / count).
// One copy per device, held until the process ends.  Host code never passes this name to a
// kernel: its device address comes from hipGetSymbolAddress, once per device.
constexpr int MSE_SCRATCH_DOUBLES = 2 * 1024 + 1;
static __device__ __align__(256) double scratch[MSE_SCRATCH_DOUBLES];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[MAX_DEVICES];

// device address of `scratch` on the current device (nullptr and *err set on failure)
static double* scratch_address(int* err)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        *err = -4;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            *err = -4;
            return nullptr;
        }
        g_scratch_ptr[dev] = static_cast<double*>(ptr);
    }
    return g_scratch_ptr[dev];
}

int lbm_cnn_masked_mse_noalloc(const float* pred, const float* target, const float* fluid, int B,
                               int C, int H, int W, float* grad, double* loss_out, void* stream)
{
    if (!pred || !target || !fluid || !grad || !loss_out || B <= 0 || C <= 0 || H <= 0 || W <= 0)
        return -1;
    const long long n = (long long)B * C * H * W;
    const int g = grid_for(n, 256, 1024);
    // pass 1 writes 2 g partial sums, pass 2 one more value: the fixed scratch must hold them
    if (2 * (long long)g + 1 > MSE_SCRATCH_DOUBLES) return -8;
    int err = 0;
    double* part = scratch_address(&err);
    if (!part) return err;
    hipStream_t st = (hipStream_t)stream;
    // every slot that pass 2 reads is written by pass 1 of this call: nothing to clear
    hipLaunchKernelGGL(k_masked_mse, dim3(g), dim3(256), 0, st, pred, target, fluid, B, C, H, W,
                       grad, part);
    int e = status(hipGetLastError());
    if (e) return e;
    hipLaunchKernelGGL(k_mse_finalize, dim3(1), dim3(64), 0, st, part, g, loss_out, part + 2 * 1024);
    e = status(hipGetLastError());
    if (e) return e;
    hipLaunchKernelGGL(k_scale, dim3(grid_for(n)), dim3(256), 0, st, grad, n, part + 2 * 1024);
    return status(hipGetLastError());
}

int lbm_cnn_adam(float* param, const float* grad, float* m, float* v, int64_t n, float lr,
                 float beta1, float beta2, float eps, int t, void* stream)
{
    if (!param || !grad || !m || !v || n < 0 || t < 1) return -1;
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, param, grad, m,
                       v, (long long)n, lr, beta1, beta2, eps, c1, c2);
    return status(hipGetLastError());
}

int lbm_cnn_to_bf16(const float* in, uint16_t* out, int64_t n, void* stream)
{
    if (!in || !out) return -1;
    hipLaunchKernelGGL(k_to_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, in, out, (long long)n);
    return status(hipGetLastError());
}

int lbm_cnn_from_bf16(const uint16_t* in, float* out, int64_t n, void* stream)
{
    if (!in || !out) return -1;
    hipLaunchKernelGGL(k_from_bf16, dim3(grid_for(n)), dim3(256), 0, (hipStream_t)stream, in, out, (long long)n);
    return status(hipGetLastError());
}

int lbm_cnn_features(const uint8_t* solid, const double* X_in, const double* j_A_cm2,
                     const double* prof, int B, int H, int W, float* feat, double* base,
                     void* stream)
{
    if (!solid || !X_in || !j_A_cm2 || !prof || !feat || !base || B <= 0 || H <= 0 || W <= 0 ||
        W > FEAT_MAX_W || B > 65535)
        return -1;
    const dim3 grid((H + FEAT_ROWS - 1) / FEAT_ROWS, B);
    const size_t lds = 2 * ((W + 1) / 2) * sizeof(int) + 2 * W * sizeof(double);
    hipLaunchKernelGGL(k_features, grid, dim3(256), lds, (hipStream_t)stream, solid, X_in,
                       j_A_cm2, prof, H, W, feat, base);
    return status(hipGetLastError());
}

int lbm_cnn_assemble(const float* pred, const double* prof, int B, int H, int W, float scale,
                     double x_min, double* X, void* stream)
{
    if (!pred || !prof || !X || B <= 0 || H <= 0 || W <= 0 || !(x_min > 0.0 && x_min < 1.0 / 3.0))
        return -1;
    hipLaunchKernelGGL(k_assemble, dim3(grid_for((long long)B * H * W)), dim3(256), 0,
                       (hipStream_t)stream, pred, prof, B, H, W, scale, x_min, X);
    return status(hipGetLastError());
}

}  // extern "C"
