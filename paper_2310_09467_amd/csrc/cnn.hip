// cnn.hip -- learned arrangement selector: band features, BF16 MFMA layers,
// softmax cross-entropy and AdamW.
//
// The selector predicts, per band, which arrangement the entropy judgement
// (paper Sec. 2.1.2) would pick, so that confident bands build only that one
// arrangement; the paper names a faster criterion as future work (Sec. 4).
//
// Features (per band, 64 x 64 cells over the band's pixel grid, area pooled):
// log1p(mean), log1p(variance), log1p(mean |x - x one lens to the left|)
// (0 in the first lens column) and log1p(mean |cur - prev|) (0 without a
// previous frame), stored channels-last [band][64][64][4].
//
// Network: conv3x3 stride 2 pad 1, 4->32, ReLU; 32->32, ReLU; 32->32, ReLU
// (64 -> 32 -> 16 -> 8); flatten 2048 -> FC 64, ReLU -> FC 4.  Weights are kept
// in FP32 (master copy for AdamW) and BF16 (GEMM operand); every layer input
// (activations, upstream gradients) is rounded to BF16; products accumulate in
// FP32 on the matrix cores (v_mfma_f32_16x16x32_bf16).  Convolutions are
// explicit im2col GEMMs: rows (image, y, x), columns (ky, kx, channel).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "pcbz.h"
#include "pcbz_internal.hpp"

namespace pcbz {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short bf16x8 __attribute__((ext_vector_type(8)));  // BF16 bits
typedef __bf16 mfma_bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16 x 16 x 32 product on the matrix cores: lane l holds row (A) or
// column (B) l % 16 and k = 8 * (l / 16) .. + 7 of the step; the result's
// element t of lane l is row 4 * (l / 16) + t, column l % 16.
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(mfma_bf16x8, a),
                                                  __builtin_bit_cast(mfma_bf16x8, b), c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 join(bf16x4 lo, bf16x4 hi) {
  return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7);
}

// Round to nearest even; NaN stays NaN.
__device__ __forceinline__ uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------- GEMM
// C(m,n) = sum_k A(m,k) B(k,n), A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]
// (BF16 bits), out-of-range elements read as zero.  One wavefront owns a
// 32 x 32 output tile (2 x 2 MFMA tiles); a workgroup of four covers 64 x 64.
// gridDim.z splits K: slice z writes C + z*split_stride (summed later).
__global__ __launch_bounds__(256) void k_gemm_bf16(int M, int N, int K, const uint16_t *A, long sam, long sak,
                                                   const uint16_t *B, long sbk, long sbn, float *C, long scm,
                                                   long scn, int ksplit_len, long split_stride) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int m0 = blockIdx.y * 64 + (w >> 1) * 32, n0 = blockIdx.x * 64 + (w & 1) * 32;
  const int kbeg = blockIdx.z * ksplit_len, kend = min(K, kbeg + ksplit_len);
  const int r = lane & 15, q = lane >> 4;  // row/column in a 16-tile, and the lane's K quarter
  f32x4 acc[2][2];
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
    bf16x8 a[2], b[2];
    for (int i = 0; i < 2; i++) {
      const int m = m0 + 16 * i + r;
      for (int j = 0; j < 8; j++) {
        const int k = k0 + 8 * q + j;
        a[i][j] = (m < M && k < kend) ? (short)A[(long)m * sam + (long)k * sak] : (short)0;
      }
    }
    for (int i = 0; i < 2; i++) {
      const int n = n0 + 16 * i + r;
      for (int j = 0; j < 8; j++) {
        const int k = k0 + 8 * q + j;
        b[i][j] = (n < N && k < kend) ? (short)B[(long)k * sbk + (long)n * sbn] : (short)0;
      }
    }
    for (int i = 0; i < 2; i++)
      for (int j = 0; j < 2; j++) acc[i][j] = mfma32(a[i], b[j], acc[i][j]);
  }
  float *Cz = C + blockIdx.z * split_stride;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++)
      for (int t = 0; t < 4; t++) {
        const int m = m0 + 16 * i + 4 * q + t, n = n0 + 16 * j + r;
        if (m < M && n < N) Cz[(long)m * scm + (long)n * scn] = acc[i][j][t];
      }
}

// out[i] = sum over z of parts[z*stride + i] (fixed order: deterministic)
__global__ void k_sum_splits(const float *parts, int nz, long stride, long n, float *out) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int z = 0; z < nz; z++) s += parts[z * stride + i];
    out[i] = s;
  }
}

// ---------------------------------------------------------------- layers
// im2col for 3x3 stride-2 pad-1 convolution, NHWC input [B][H][W][C] (BF16).
__global__ void k_im2col(const uint16_t *x, int B, int H, int W, int C, uint16_t *col) {
  const int Ho = H / 2, Wo = W / 2, K = 9 * C;
  const long total = (long)B * Ho * Wo * K;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int k = (int)(i % K);
    const long m = i / K;
    const int ox = (int)(m % Wo), oy = (int)((m / Wo) % Ho), b = (int)(m / ((long)Wo * Ho));
    const int c = k % C, kx = (k / C) % 3, ky = k / (3 * C);
    const int y = 2 * oy - 1 + ky, xx = 2 * ox - 1 + kx;
    col[i] = (y >= 0 && y < H && xx >= 0 && xx < W) ? x[(((long)b * H + y) * W + xx) * C + c] : (uint16_t)0;
  }
}

// Gradient of im2col: dx(b,y,x,c) = sum of dcol over the (ky,kx) that read it.
__global__ void k_col2im(const float *dcol, int B, int H, int W, int C, float *dx) {
  const int Ho = H / 2, Wo = W / 2, K = 9 * C;
  const long total = (long)B * H * W * C;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const int xx = (int)((i / C) % W), y = (int)((i / ((long)C * W)) % H), b = (int)(i / ((long)C * W * H));
    float s = 0.f;
    for (int ky = 0; ky < 3; ky++) {
      const int ty = y + 1 - ky;
      if (ty < 0 || (ty & 1) || ty / 2 >= Ho) continue;
      for (int kx = 0; kx < 3; kx++) {
        const int tx = xx + 1 - kx;
        if (tx < 0 || (tx & 1) || tx / 2 >= Wo) continue;
        const long m = ((long)b * Ho + ty / 2) * Wo + tx / 2;
        s += dcol[m * K + (ky * 3 + kx) * C + c];
      }
    }
    dx[i] = s;
  }
}

// y = act(acc + bias) -> FP32 pre-activation kept for backward, BF16 output.
__global__ void k_bias_act(const float *acc, const float *bias, long M, int N, int relu, float *pre, uint16_t *out16,
                           float *out32) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < M * N; i += (long)gridDim.x * blockDim.x) {
    const float v = acc[i] + bias[i % N];
    if (pre) pre[i] = v;
    const float a = relu ? fmaxf(v, 0.f) : v;
    if (out16) out16[i] = f2bf(a);
    if (out32) out32[i] = a;
  }
}

// g16 = bf16(g * (pre > 0)) for the backward of a ReLU layer (or no mask)
__global__ void k_relu_grad(const float *g, const float *pre, long n, uint16_t *g16) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    g16[i] = f2bf(pre && pre[i] <= 0.f ? 0.f : g[i]);
}

// db[n] = sum over rows of g[m][n] (bf16 gradient values as used by the GEMMs)
__global__ void k_bias_grad(const uint16_t *g16, long M, int N, float *db) {
  const int n = blockIdx.x;
  float s = 0.f;
  for (long m = threadIdx.x; m < M; m += blockDim.x) s += bf2f(g16[m * N + n]);
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[n] = red[0];
}

// Softmax cross-entropy with class weights, mean over the batch weighted by
// w[label]: loss = sum_i w_i * (-log p_i[label_i]) / sum_i w_i.
// Labels above 3 set *err and are read as 3.
__global__ void k_softmax_ce(const float *logits, const uint8_t *label, const float *cw, int n, float *dlogits,
                             float *loss_out, uint32_t *err) {
  __shared__ float red[2][256];
  float lsum = 0.f, wsum = 0.f;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float *z = logits + 4 * i;
    const float mx = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
    const float e0 = expf(z[0] - mx), e1 = expf(z[1] - mx), e2 = expf(z[2] - mx), e3 = expf(z[3] - mx);
    const float se = e0 + e1 + e2 + e3;
    if (label[i] > 3) atomicOr(err, 1u);
    const int y = min((int)label[i], 3);
    const float wy = cw[y];
    lsum += wy * (logf(se) - (z[y] - mx));
    wsum += wy;
  }
  red[0][threadIdx.x] = lsum;
  red[1][threadIdx.x] = wsum;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) {
      red[0][threadIdx.x] += red[0][threadIdx.x + d];
      red[1][threadIdx.x] += red[1][threadIdx.x + d];
    }
    __syncthreads();
  }
  const float W = red[1][0];
  if (threadIdx.x == 0 && loss_out) *loss_out = red[0][0] / W;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const float *z = logits + 4 * i;
    const float mx = fmaxf(fmaxf(z[0], z[1]), fmaxf(z[2], z[3]));
    float e[4];
    float se = 0.f;
    for (int c = 0; c < 4; c++) {
      e[c] = expf(z[c] - mx);
      se += e[c];
    }
    const int y = min((int)label[i], 3);
    const float s = cw[y] / W;
    for (int c = 0; c < 4; c++) dlogits[4 * i + c] = s * (e[c] / se - (c == y ? 1.f : 0.f));
  }
}

// AdamW on the FP32 master copy; the BF16 copy follows.
__global__ void k_adamw(float *p, float *m, float *v, const float *g, uint16_t *p16, long n, float lr, float b1,
                        float b2, float eps, float wd, float c1, float c2) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float upd = (mi / c1) / (sqrtf(vi / c2) + eps);
    const float pi = p[i] * (1.f - lr * wd) - lr * upd;
    p[i] = pi;
    p16[i] = f2bf(pi);
  }
}

__global__ void k_to_bf16(const float *x, long n, uint16_t *y) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) y[i] = f2bf(x[i]);
}

// Normalised network input: bf16((f - mean[c]) / std[c]), channels last.
__global__ void k_norm_input(const float *f, long n, const float *mean, const float *stdv, uint16_t *x) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const int c = (int)(i & 3);
    x[i] = f2bf((f[i] - mean[c]) / stdv[c]);
  }
}

// ---------------------------------------------------------------- features
// One workgroup per (cell row, band).  Threads walk pixel columns (coalesced
// row reads) and sum each column's pixels of the cell row exactly in
// integers, then add the column sums into the column's cell in LDS; 64
// threads finish the cells.  The integer sums equal the double sums of the
// definition, so the results are the same.
__global__ __launch_bounds__(256) void k_features(const BandDesc *bands, uint32_t n_bands, float *feat) {
  __shared__ unsigned long long s_sum[64], s_sq[64], s_dx[64], s_dt[64];
  const uint32_t ci = blockIdx.x, b = blockIdx.y;
  if (b >= n_bands) return;
  const BandDesc B = bands[b];
  const uint32_t Hb = B.Rb * B.pitch, W = B.W, p = B.pitch;
  const uint32_t y0 = ci * Hb / 64, y1 = (ci + 1) * Hb / 64;
  if (threadIdx.x < 64) {
    s_sum[threadIdx.x] = 0;
    s_sq[threadIdx.x] = 0;
    s_dx[threadIdx.x] = 0;
    s_dt[threadIdx.x] = 0;
  }
  __syncthreads();
  for (uint32_t x = threadIdx.x; x < W; x += blockDim.x) {
    unsigned long long sum = 0, sq = 0, dx = 0, dt = 0;
    for (uint32_t y = y0; y < y1; y++) {
      const size_t o = (size_t)(B.y0 + y) * W + x;
      const uint32_t v = B.frame[o];
      sum += v;
      sq += (unsigned long long)v * v;
      if (x >= p) dx += (uint32_t)abs((int)v - (int)B.frame[o - p]);
      if (B.prev) dt += (uint32_t)abs((int)v - (int)B.prev[o]);
    }
    if (y1 > y0) {
      // cell j covers columns [j*W/64, (j+1)*W/64)
      const uint32_t j = min(63u, (uint32_t)(((uint64_t)x * 64 + 63) / W));
      atomicAdd(&s_sum[j], sum);
      atomicAdd(&s_sq[j], sq);
      atomicAdd(&s_dx[j], dx);
      atomicAdd(&s_dt[j], dt);
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint32_t cj = threadIdx.x;
    const uint32_t x0 = cj * W / 64, x1 = (cj + 1) * W / 64;
    const uint32_t cnt = (y1 - y0) * (x1 - x0);
    float *o = feat + ((size_t)b * 4096 + ci * 64 + cj) * 4;
    if (cnt == 0) {
      o[0] = o[1] = o[2] = o[3] = 0.f;
    } else {
      const double mean = (double)s_sum[cj] / cnt, var = fmax((double)s_sq[cj] / cnt - mean * mean, 0.0);
      o[0] = (float)log1p(mean);
      o[1] = (float)log1p(var);
      o[2] = (float)log1p((double)s_dx[cj] / cnt);
      o[3] = (float)log1p((double)s_dt[cj] / cnt);
    }
  }
}

// ---------------------------------------------------------------- fused inference
// The whole network for one band per workgroup (four wavefronts), with every
// activation in LDS.  Convolutions are tiles of 16 output pixels x 16
// channels on the matrix cores; a lane's A operand is eight consecutive
// entries of the im2col row (two runs of four channels of one input pixel,
// one 8-byte LDS read each) and its B operand eight consecutive weights of
// one output channel.  The fully connected layers use the same instruction
// with the sample in row 0.  K is walked in steps of 32 in the same order as
// the layer-by-layer path, so both give the same logits.
template <int H, int C>
__device__ __forceinline__ void conv_tile_layer(const uint16_t *X, const uint16_t *Wt, const float *bias,
                                                uint16_t *Y) {
  constexpr int Ho = H / 2, M = Ho * Ho, K = 9 * C, KS = (K + 31) / 32;
  static_assert(C % 4 == 0, "a run of four channels stays in one pixel");
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int r = lane & 15, q = lane >> 4;
  for (int mt = w; mt < M / 16; mt += 4) {
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    const int m = mt * 16 + r, oy = m / Ho, ox = m % Ho;
    for (int ks = 0; ks < KS; ks++) {
      bf16x4 a[2], b0[2], b1[2];
#pragma unroll
      for (int hf = 0; hf < 2; hf++) {
        const int k0 = ks * 32 + 8 * q + 4 * hf;  // this lane's run of four k
        a[hf] = b0[hf] = b1[hf] = bf16x4{0, 0, 0, 0};
        if (k0 < K) {
          const int pos = k0 / C, c0 = k0 % C, ky = pos / 3, kx = pos % 3;
          const int iy = 2 * oy - 1 + ky, ix = 2 * ox - 1 + kx;
          if (iy >= 0 && iy < H && ix >= 0 && ix < H) a[hf] = *(const bf16x4 *)(X + (iy * H + ix) * C + c0);
          b0[hf] = *(const bf16x4 *)(Wt + (size_t)r * K + k0);
          b1[hf] = *(const bf16x4 *)(Wt + (size_t)(16 + r) * K + k0);
        }
      }
      const bf16x8 av = join(a[0], a[1]);
      acc0 = mfma32(av, join(b0[0], b0[1]), acc0);
      acc1 = mfma32(av, join(b1[0], b1[1]), acc1);
    }
#pragma unroll
    for (int j = 0; j < 4; j++) {
      const int mo = mt * 16 + 4 * q + j;
      Y[mo * 32 + r] = f2bf(fmaxf(acc0[j] + bias[r], 0.f));
      Y[mo * 32 + 16 + r] = f2bf(fmaxf(acc1[j] + bias[16 + r], 0.f));
    }
  }
}

// out = W x (+ bias, ReLU to bf16 or plain FP32) for one sample: x has K
// entries, W is [N][K]; wavefront w computes outputs [16w, 16w + 16).
template <int K, int N>
__device__ __forceinline__ void fc_layer(const uint16_t *x, const uint16_t *Wt, const float *bias, uint16_t *out16,
                                         float *out32) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const int r = lane & 15, q = lane >> 4;
  if (w * 16 >= N) return;
  static_assert(K % 32 == 0, "whole steps of 32");
  const int n = w * 16 + r;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 8 * q; k0 < K; k0 += 32) {
    bf16x8 a = {0, 0, 0, 0, 0, 0, 0, 0}, b = {0, 0, 0, 0, 0, 0, 0, 0};
    if (r == 0) a = join(*(const bf16x4 *)(x + k0), *(const bf16x4 *)(x + k0 + 4));
    if (n < N) b = join(*(const bf16x4 *)(Wt + (size_t)n * K + k0), *(const bf16x4 *)(Wt + (size_t)n * K + k0 + 4));
    acc = mfma32(a, b, acc);
  }
  // row 0 of the result sits in lanes 0..15, element 0
  if (q == 0 && n < N) {
    const float v = acc[0] + bias[n];
    if (out16) out16[n] = f2bf(fmaxf(v, 0.f));
    if (out32) out32[n] = v;
  }
}

__global__ __launch_bounds__(256) void k_sel_infer(const float *feat, const float *norm, const uint16_t *p16,
                                                   const float *p, long oW1, long oB1, long oW2, long oB2, long oW3,
                                                   long oB3, long oW4, long oB4, long oW5, long oB5,
                                                   float *logits) {
  __shared__ __align__(16) uint16_t bufA[64 * 64 * 4];    // x0, then x2
  __shared__ __align__(16) uint16_t bufB[32 * 32 * 32];   // x1, then x3
  __shared__ __align__(16) uint16_t x4[64];
  __shared__ __align__(16) uint32_t sW[32 * 288 / 2];     // one conv layer's weights
  const size_t sample = blockIdx.x;
  const float *f = feat + sample * 16384;
  for (int i = threadIdx.x; i < 16384; i += 256) {
    const int c = i & 3;
    bufA[i] = f2bf((f[i] - norm[c]) / norm[4 + c]);
  }
  stage_to_lds(sW, (const uint32_t *)(p16 + oW1), 32 * 36 / 2);
  __syncthreads();
  conv_tile_layer<64, 4>(bufA, (const uint16_t *)sW, p + oB1, bufB);
  __syncthreads();
  stage_to_lds(sW, (const uint32_t *)(p16 + oW2), 32 * 288 / 2);
  __syncthreads();
  conv_tile_layer<32, 32>(bufB, (const uint16_t *)sW, p + oB2, bufA);
  __syncthreads();
  stage_to_lds(sW, (const uint32_t *)(p16 + oW3), 32 * 288 / 2);
  __syncthreads();
  conv_tile_layer<16, 32>(bufA, (const uint16_t *)sW, p + oB3, bufB);
  __syncthreads();
  fc_layer<2048, 64>(bufB, p16 + oW4, p + oB4, x4, nullptr);
  __syncthreads();
  fc_layer<64, 4>(x4, p16 + oW5, p + oB5, nullptr, logits + sample * 4);
}

// Confident bands get the network's choice; the rest (p_max < min_conf) are
// left to the entropy judgement (0xFF).  Counts the fallbacks.
__global__ void k_select(const float *logits, uint32_t n_bands, const BandDesc *bands, float min_conf,
                         uint8_t *forced, uint32_t *n_fallback) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bands) return;
  if (forced[b] != 0xFFu) return;  // the caller forced this band
  const float *z = logits + 4 * b;
  const uint32_t mask = bands[b].cand_mask;
  if (mask >> kNumBasic) {  // the network predicts ids 0..3 only: bands offering the predictor family are judged
    atomicAdd(n_fallback, 1u);
    return;
  }
  float mx = -INFINITY;
  int best = -1;
  for (int c = 0; c < 4; c++)
    if ((mask >> c) & 1u)
      if (best < 0 || z[c] > mx) {
        mx = z[c];
        best = c;
      }
  float se = 0.f;
  for (int c = 0; c < 4; c++)
    if ((mask >> c) & 1u) se += expf(z[c] - mx);
  const float pmax = 1.f / se;
  if (best >= 0 && pmax >= min_conf)
    forced[b] = (uint8_t)best;
  else
    atomicAdd(n_fallback, 1u);
}

uint32_t grid1(long n) {
  long g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 8192) g = 8192;
  return (uint32_t)g;
}

}  // namespace

// ---------------------------------------------------------------- host side
void gemm_bf16(int M, int N, int K, const uint16_t *A, long sam, long sak, const uint16_t *B, long sbk, long sbn,
               float *C, long scm, long scn, float *split_tmp, hipStream_t s) {
  // split long reductions so that enough workgroups run; parts summed in order
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int nz = 1;
  if (split_tmp && K >= 4096 && tiles < 256) {
    nz = (int)std::min<long>(64, std::max<long>(1, K / 2048));
    while (nz > 1 && (long)nz * M * N > (long)16 << 20) nz--;
  }
  const int klen = ((K + nz - 1) / nz + 31) / 32 * 32;  // whole steps of the matrix-core product
  nz = (K + klen - 1) / klen;
  dim3 grid((N + 63) / 64, (M + 63) / 64, nz);
  if (nz == 1) {
    PCBZ_LAUNCH(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, C, scm, scn, klen, 0l);
    return;
  }
  // parts in a dense M x N layout, then summed into C (dense, scn == 1, scm == N)
  PCBZ_LAUNCH(k_gemm_bf16, grid, dim3(256), 0, s, M, N, K, A, sam, sak, B, sbk, sbn, split_tmp, (long)N, 1l, klen,
              (long)M * N);
  PCBZ_LAUNCH(k_sum_splits, dim3(grid1((long)M * N)), dim3(256), 0, s, split_tmp, nz, (long)M * N, (long)M * N, C);
  (void)scm;
  (void)scn;
}

// ---------------------------------------------------------------- selector
namespace {
// Parameter layout (FP32 master copy, in this order).
constexpr long kW1 = 0, kB1 = kW1 + 32 * 9 * 4;
constexpr long kW2 = kB1 + 32, kB2 = kW2 + 32 * 9 * 32;
constexpr long kW3 = kB2 + 32, kB3 = kW3 + 32 * 9 * 32;
constexpr long kW4 = kB3 + 32, kB4 = kW4 + 64 * 2048;
constexpr long kW5 = kB4 + 64, kB5 = kW5 + 4 * 64;
constexpr long kNumParams = kB5 + 4;
}  // namespace

long selector_num_params() { return kNumParams; }

struct SelWork {
  uint32_t cap = 0;
  uint16_t *x0 = nullptr, *col1 = nullptr, *x1 = nullptr, *col2 = nullptr, *x2 = nullptr, *col3 = nullptr,
           *x3 = nullptr, *x4 = nullptr, *g16 = nullptr;
  float *acc = nullptr, *pre1 = nullptr, *pre2 = nullptr, *pre3 = nullptr, *pre4 = nullptr, *logits = nullptr,
        *dlog = nullptr, *dx = nullptr, *dcol = nullptr, *split = nullptr, *loss = nullptr, *cw = nullptr;
  uint32_t *err = nullptr;
  uint32_t last_n = 0;  // samples of the last gradients call (0: none yet)
};

// The backward pass keeps each layer's bf16 gradient (dL/dpre after the ReLU
// mask) in its own slice of g16, so a finished call can be inspected layer by
// layer: per sample 4 (FC5), 64 (FC4), 64x32 (conv3), 256x32 (conv2),
// 1024x32 (conv1) values.
constexpr long kG16Sample = 4 + 64 + 2048 + 8192 + 32768;
inline uint16_t *g16_layer(const SelWork &w, int layer, long n) {
  long off = 0;
  const long per[6] = {0, 32768, 8192, 2048, 64, 4};  // by layer 1..5
  for (int l = 5; l > layer; l--) off += per[l] * n;
  return w.g16 + off;
}

}  // namespace pcbz

struct pcbz_selector {
  int device = 0;
  float *p = nullptr, *m = nullptr, *v = nullptr, *g = nullptr;
  uint16_t *p16 = nullptr;
  float norm[8] = {0, 0, 0, 0, 1, 1, 1, 1};  // mean[4], std[4]
  float *d_norm = nullptr;
  long step = 0;
  uint64_t gen = 1;  // bumped when the workspace moves
  pcbz::SelWork w;
};

namespace pcbz {
namespace {

template <typename T>
hipError_t dalloc(T **p, size_t n) {
  return hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
}

void free_work(SelWork &w) {
  void *ptrs[] = {w.x0, w.col1, w.x1, w.col2, w.x2, w.col3, w.x3, w.x4, w.g16, w.acc, w.pre1, w.pre2, w.pre3,
                  w.pre4, w.logits, w.dlog, w.dx, w.dcol, w.split, w.loss, w.cw, w.err};
  for (void *q : ptrs)
    if (q) (void)hipFree(q);
  w = SelWork();
}

int ensure_work(pcbz_selector *S, uint32_t n) {
  SelWork &w = S->w;
  if (n <= w.cap) return PCBZ_OK;
  (void)hipDeviceSynchronize();
  free_work(w);
  const size_t N = n;
  hipError_t e = hipSuccess;
  auto A = [&](hipError_t r) {
    if (r != hipSuccess) e = r;
  };
  A(dalloc(&w.x0, N * 4096 * 4));
  A(dalloc(&w.col1, N * 1024 * 36));
  A(dalloc(&w.x1, N * 1024 * 32));
  A(dalloc(&w.col2, N * 256 * 288));
  A(dalloc(&w.x2, N * 256 * 32));
  A(dalloc(&w.col3, N * 64 * 288));
  A(dalloc(&w.x3, N * 2048));
  A(dalloc(&w.x4, N * 64));
  A(dalloc(&w.g16, N * kG16Sample));
  A(dalloc(&w.acc, N * 1024 * 32));
  A(dalloc(&w.pre1, N * 1024 * 32));
  A(dalloc(&w.pre2, N * 256 * 32));
  A(dalloc(&w.pre3, N * 64 * 32));
  A(dalloc(&w.pre4, N * 64));
  A(dalloc(&w.logits, N * 4));
  A(dalloc(&w.dlog, N * 4));
  A(dalloc(&w.dx, N * 1024 * 32));
  A(dalloc(&w.dcol, N * 256 * 288));
  A(dalloc(&w.split, (size_t)16 << 20));
  A(dalloc(&w.loss, 4));
  A(dalloc(&w.cw, 4));
  A(dalloc(&w.err, 1));
  if (e != hipSuccess) {
    free_work(w);
    return PCBZ_ENOMEM;
  }
  w.cap = n;
  S->gen++;
  return PCBZ_OK;
}

void conv_forward(const uint16_t *x, int n, int H, int C, const uint16_t *W16, const float *bias, uint16_t *col,
                  float *acc, float *pre, uint16_t *y, hipStream_t s) {
  const long M = (long)n * (H / 2) * (H / 2);
  const int K = 9 * C;
  PCBZ_LAUNCH(k_im2col, dim3(grid1(M * K)), dim3(256), 0, s, x, n, H, H, C, col);
  gemm_bf16((int)M, 32, K, col, K, 1, W16, 1, K, acc, 32, 1, nullptr, s);
  PCBZ_LAUNCH(k_bias_act, dim3(grid1(M * 32)), dim3(256), 0, s, acc, bias, M, 32, 1, pre, y, (float *)nullptr);
}

// Forward pass for n samples of features [n][64][64][4]; logits in w.logits.
void forward(pcbz_selector *S, const float *feat, uint32_t n, hipStream_t s) {
  SelWork &w = S->w;
  const long n0 = (long)n * 4096 * 4;
  PCBZ_LAUNCH(k_norm_input, dim3(grid1(n0)), dim3(256), 0, s, feat, n0, S->d_norm, S->d_norm + 4, w.x0);
  conv_forward(w.x0, n, 64, 4, S->p16 + kW1, S->p + kB1, w.col1, w.acc, w.pre1, w.x1, s);
  conv_forward(w.x1, n, 32, 32, S->p16 + kW2, S->p + kB2, w.col2, w.acc, w.pre2, w.x2, s);
  conv_forward(w.x2, n, 16, 32, S->p16 + kW3, S->p + kB3, w.col3, w.acc, w.pre3, w.x3, s);
  gemm_bf16((int)n, 64, 2048, w.x3, 2048, 1, S->p16 + kW4, 1, 2048, w.acc, 64, 1, nullptr, s);
  PCBZ_LAUNCH(k_bias_act, dim3(grid1((long)n * 64)), dim3(256), 0, s, w.acc, S->p + kB4, (long)n, 64, 1, w.pre4, w.x4,
              (float *)nullptr);
  gemm_bf16((int)n, 4, 64, w.x4, 64, 1, S->p16 + kW5, 1, 64, w.acc, 4, 1, nullptr, s);
  PCBZ_LAUNCH(k_bias_act, dim3(grid1((long)n * 4)), dim3(256), 0, s, w.acc, S->p + kB5, (long)n, 4, 0,
              (float *)nullptr, (uint16_t *)nullptr, w.logits);
}

// Backward of a conv layer: g16 holds bf16(dL/dpre) [M][32]; writes dW, db and
// (if dx) the gradient of the layer input (FP32, before the lower ReLU).
void conv_backward(int n, int H, int C, const uint16_t *col, const uint16_t *g16, const uint16_t *W16, float *dW,
                   float *db, float *dcol, float *dx, float *split, hipStream_t s) {
  const long M = (long)n * (H / 2) * (H / 2);
  const int K = 9 * C;
  gemm_bf16(32, K, (int)M, g16, 1, 32, col, K, 1, dW, K, 1, split, s);
  PCBZ_LAUNCH(k_bias_grad, dim3(32), dim3(256), 0, s, g16, M, 32, db);
  if (dx) {
    gemm_bf16((int)M, K, 32, g16, 32, 1, W16, K, 1, dcol, K, 1, nullptr, s);
    PCBZ_LAUNCH(k_col2im, dim3(grid1((long)n * H * H * C)), dim3(256), 0, s, dcol, n, H, H, C, dx);
  }
}

// Backward from w.dlog; gradients into S->g.
void backward(pcbz_selector *S, uint32_t n, hipStream_t s) {
  SelWork &w = S->w;
  float *g = S->g;
  uint16_t *g5 = g16_layer(w, 5, n), *g4 = g16_layer(w, 4, n), *g3 = g16_layer(w, 3, n), *g2 = g16_layer(w, 2, n),
           *g1 = g16_layer(w, 1, n);
  // FC 64 -> 4 (no activation)
  PCBZ_LAUNCH(k_relu_grad, dim3(grid1((long)n * 4)), dim3(256), 0, s, w.dlog, (const float *)nullptr, (long)n * 4, g5);
  gemm_bf16(4, 64, (int)n, g5, 1, 4, w.x4, 64, 1, g + kW5, 64, 1, w.split, s);
  PCBZ_LAUNCH(k_bias_grad, dim3(4), dim3(256), 0, s, g5, (long)n, 4, g + kB5);
  gemm_bf16((int)n, 64, 4, g5, 4, 1, S->p16 + kW5, 64, 1, w.dx, 64, 1, nullptr, s);
  // FC 2048 -> 64, ReLU
  PCBZ_LAUNCH(k_relu_grad, dim3(grid1((long)n * 64)), dim3(256), 0, s, w.dx, w.pre4, (long)n * 64, g4);
  gemm_bf16(64, 2048, (int)n, g4, 1, 64, w.x3, 2048, 1, g + kW4, 2048, 1, w.split, s);
  PCBZ_LAUNCH(k_bias_grad, dim3(64), dim3(256), 0, s, g4, (long)n, 64, g + kB4);
  gemm_bf16((int)n, 2048, 64, g4, 64, 1, S->p16 + kW4, 2048, 1, w.dx, 2048, 1, nullptr, s);
  // conv3 (16 -> 8), input x2
  PCBZ_LAUNCH(k_relu_grad, dim3(grid1((long)n * 2048)), dim3(256), 0, s, w.dx, w.pre3, (long)n * 2048, g3);
  conv_backward((int)n, 16, 32, w.col3, g3, S->p16 + kW3, g + kW3, g + kB3, w.dcol, w.dx, w.split, s);
  // conv2 (32 -> 16), input x1
  PCBZ_LAUNCH(k_relu_grad, dim3(grid1((long)n * 8192)), dim3(256), 0, s, w.dx, w.pre2, (long)n * 8192, g2);
  conv_backward((int)n, 32, 32, w.col2, g2, S->p16 + kW2, g + kW2, g + kB2, w.dcol, w.dx, w.split, s);
  // conv1 (64 -> 32), input x0: no input gradient
  PCBZ_LAUNCH(k_relu_grad, dim3(grid1((long)n * 32768)), dim3(256), 0, s, w.dx, w.pre1, (long)n * 32768, g1);
  conv_backward((int)n, 64, 4, w.col1, g1, S->p16 + kW1, g + kW1, g + kB1, w.dcol, (float *)nullptr, w.split, s);
}

int upload_params(pcbz_selector *S, const float *host) {
  if (hipMemcpy(S->p, host, kNumParams * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) return PCBZ_EDEVICE;
  PCBZ_LAUNCH(k_to_bf16, dim3(grid1(kNumParams)), dim3(256), 0, nullptr, S->p, kNumParams, S->p16);
  if (hipMemcpy(S->d_norm, S->norm, sizeof S->norm, hipMemcpyHostToDevice) != hipSuccess) return PCBZ_EDEVICE;
  if (hipDeviceSynchronize() != hipSuccess) return PCBZ_EDEVICE;
  return PCBZ_OK;
}

}  // namespace

uint64_t selector_gen(const pcbz_selector *S) { return S->gen; }

int selector_forward(pcbz_selector *S, const float *feat, uint32_t n, float *logits, hipStream_t s) {
  if (!n) return PCBZ_OK;
  PCBZ_LAUNCH(k_sel_infer, dim3(n), dim3(256), 0, s, feat, S->d_norm, S->p16, S->p, kW1, kB1, kW2, kB2, kW3, kB3,
              kW4, kB4, kW5, kB5, logits);
  return PCBZ_OK;
}

void launch_features(const BandDesc *bands, uint32_t n_bands, float *feat, hipStream_t s) {
  if (!n_bands) return;
  PCBZ_LAUNCH(k_features, dim3(64, n_bands), dim3(256), 0, s, bands, n_bands, feat);
}

void launch_select(const float *logits, uint32_t n_bands, const BandDesc *bands, float min_conf, uint8_t *forced,
                   uint32_t *n_fallback, hipStream_t s) {
  if (!n_bands) return;
  PCBZ_LAUNCH(k_select, dim3((n_bands + 127) / 128), dim3(128), 0, s, logits, n_bands, bands, min_conf, forced,
              n_fallback);
}

}  // namespace pcbz

using namespace pcbz;

extern "C" {

int pcbz_selector_create(pcbz_ctx *ctx, const float *host_params, const float *norm8, pcbz_selector **out) {
  if (!ctx || !out) return PCBZ_EINVAL;
  *out = nullptr;
  pcbz_selector *S = new pcbz_selector();
  S->device = context_device(ctx);
  if (hipSetDevice(S->device) != hipSuccess) {
    delete S;
    return PCBZ_EDEVICE;
  }
  bool ok = dalloc(&S->p, kNumParams) == hipSuccess && dalloc(&S->m, kNumParams) == hipSuccess &&
            dalloc(&S->v, kNumParams) == hipSuccess && dalloc(&S->g, kNumParams) == hipSuccess &&
            dalloc(&S->p16, kNumParams) == hipSuccess && dalloc(&S->d_norm, 8) == hipSuccess;
  if (!ok) {
    pcbz_selector_free(S);
    return PCBZ_ENOMEM;
  }
  (void)hipMemset(S->m, 0, kNumParams * sizeof(float));
  (void)hipMemset(S->v, 0, kNumParams * sizeof(float));
  (void)hipMemset(S->g, 0, kNumParams * sizeof(float));
  if (norm8) memcpy(S->norm, norm8, sizeof S->norm);
  std::vector<float> zero;
  if (!host_params) zero.assign(kNumParams, 0.f);
  int st = upload_params(S, host_params ? host_params : zero.data());
  if (st) {
    pcbz_selector_free(S);
    return st;
  }
  *out = S;
  return PCBZ_OK;
}

void pcbz_selector_free(pcbz_selector *S) {
  if (!S) return;
  (void)hipDeviceSynchronize();
  free_work(S->w);
  float *f[] = {S->p, S->m, S->v, S->g, S->d_norm};
  for (float *q : f)
    if (q) (void)hipFree(q);
  if (S->p16) (void)hipFree(S->p16);
  delete S;
}

size_t pcbz_selector_num_params(void) { return (size_t)kNumParams; }

int pcbz_selector_get_params(const pcbz_selector *S, float *host, float *norm8) {
  if (!S) return PCBZ_EINVAL;
  if (host && hipMemcpy(host, S->p, kNumParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return PCBZ_EDEVICE;
  if (norm8) memcpy(norm8, S->norm, sizeof S->norm);
  return PCBZ_OK;
}

int pcbz_selector_set_params(pcbz_selector *S, const float *host, const float *norm8) {
  if (!S || !host) return PCBZ_EINVAL;
  if (norm8) memcpy(S->norm, norm8, sizeof S->norm);
  return upload_params(S, host);
}

int pcbz_selector_save(const pcbz_selector *S, const char *path) {
  if (!S || !path) return PCBZ_EINVAL;
  std::vector<float> h(kNumParams);
  if (hipMemcpy(h.data(), S->p, kNumParams * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
    return PCBZ_EDEVICE;
  FILE *f = fopen(path, "wb");
  if (!f) return PCBZ_EINVAL;
  const uint32_t np = (uint32_t)kNumParams;
  bool ok = fwrite("PCBZSEL1", 1, 8, f) == 8 && fwrite(&np, 4, 1, f) == 1 && fwrite(S->norm, 4, 8, f) == 8 &&
            fwrite(h.data(), 4, kNumParams, f) == (size_t)kNumParams;
  fclose(f);
  return ok ? PCBZ_OK : PCBZ_EINVAL;
}

int pcbz_selector_load(pcbz_ctx *ctx, const char *path, pcbz_selector **out) {
  if (!path || !out) return PCBZ_EINVAL;
  FILE *f = fopen(path, "rb");
  if (!f) return PCBZ_EINVAL;
  char magic[8];
  uint32_t np = 0;
  float norm[8];
  std::vector<float> h(kNumParams);
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, "PCBZSEL1", 8) == 0 && fread(&np, 4, 1, f) == 1 &&
            np == (uint32_t)kNumParams && fread(norm, 4, 8, f) == 8 &&
            fread(h.data(), 4, kNumParams, f) == (size_t)kNumParams;
  fclose(f);
  if (!ok) return PCBZ_EDATA;
  return pcbz_selector_create(ctx, h.data(), norm, out);
}

int pcbz_selector_forward(pcbz_selector *S, const float *d_feat, uint32_t n, float *d_logits, void *stream) {
  if (!S || !d_feat || !d_logits) return PCBZ_EINVAL;
  int st = selector_forward(S, d_feat, n, d_logits, (hipStream_t)stream);
  if (st) return st;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? PCBZ_OK : PCBZ_EDEVICE;
}

int pcbz_selector_gradients(pcbz_selector *S, const float *d_feat, const uint8_t *d_label, uint32_t n,
                            const float *class_w4, float *d_grad, float *loss, void *stream) {
  if (!S || !d_feat || !d_label || n == 0 || n > 4096) return PCBZ_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  int st = ensure_work(S, n);
  if (st) return st;
  const float one[4] = {1.f, 1.f, 1.f, 1.f};
  const uint32_t zero = 0;
  // the previous call on this selector may still read cw / err
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(S->w.cw, class_w4 ? class_w4 : one, 4 * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(S->w.err, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess)
    return PCBZ_EDEVICE;
  S->w.last_n = 0;
  forward(S, d_feat, n, s);
  PCBZ_LAUNCH(k_softmax_ce, dim3(1), dim3(256), 0, s, S->w.logits, d_label, S->w.cw, (int)n, S->w.dlog, S->w.loss,
              S->w.err);
  backward(S, n, s);
  if (d_grad && hipMemcpyAsync(d_grad, S->g, kNumParams * sizeof(float), hipMemcpyDeviceToDevice, s) != hipSuccess)
    return PCBZ_EDEVICE;
  float h_loss = 0.f;
  uint32_t h_err = 0;
  if (hipStreamSynchronize(s) != hipSuccess ||
      hipMemcpy(&h_loss, S->w.loss, sizeof h_loss, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&h_err, S->w.err, sizeof h_err, hipMemcpyDeviceToHost) != hipSuccess)
    return PCBZ_EDEVICE;
  if (loss) *loss = h_loss;
  S->w.last_n = n;
  return h_err ? PCBZ_EINVAL : PCBZ_OK;
}

int pcbz_selector_inspect(const pcbz_selector *S, int which, void *host, size_t bytes) {
  if (!S || !host || S->w.last_n == 0) return PCBZ_EINVAL;
  const SelWork &w = S->w;
  const long n = w.last_n;
  const void *src = nullptr;
  long count = 0;
  size_t elem = 2;
  switch (which) {
    case 0: src = w.x0, count = n * 16384; break;
    case 1: src = w.x1, count = n * 32768; break;
    case 2: src = w.x2, count = n * 8192; break;
    case 3: src = w.x3, count = n * 2048; break;
    case 4: src = w.x4, count = n * 64; break;
    case 5: src = w.pre1, count = n * 32768, elem = 4; break;
    case 6: src = w.pre2, count = n * 8192, elem = 4; break;
    case 7: src = w.pre3, count = n * 2048, elem = 4; break;
    case 8: src = w.pre4, count = n * 64, elem = 4; break;
    case 9: src = w.logits, count = n * 4, elem = 4; break;
    case 10: src = w.dlog, count = n * 4, elem = 4; break;
    case 11: case 12: case 13: case 14: case 15: {
      const int layer = 16 - which;  // 11 -> FC5 ... 15 -> conv1
      const long per[6] = {0, 32768, 8192, 2048, 64, 4};
      src = g16_layer(w, layer, n);
      count = per[layer] * n;
      break;
    }
    default: return PCBZ_EINVAL;
  }
  if (bytes != (size_t)count * elem) return PCBZ_EINVAL;
  if (hipSetDevice(S->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(host, src, bytes, hipMemcpyDeviceToHost) != hipSuccess)
    return PCBZ_EDEVICE;
  return PCBZ_OK;
}

int pcbz_selector_train_step(pcbz_selector *S, const float *d_feat, const uint8_t *d_label, uint32_t n,
                             const float *class_w4, float lr, float weight_decay, float *loss, void *stream) {
  int st = pcbz_selector_gradients(S, d_feat, d_label, n, class_w4, nullptr, loss, stream);
  if (st) return st;
  S->step++;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)S->step), c2 = 1.f - powf(b2, (float)S->step);
  hipStream_t s = (hipStream_t)stream;
  PCBZ_LAUNCH(k_adamw, dim3(grid1(kNumParams)), dim3(256), 0, s, S->p, S->m, S->v, S->g, S->p16, kNumParams, lr, b1,
              b2, 1e-8f, weight_decay, c1, c2);
  return hipStreamSynchronize(s) == hipSuccess ? PCBZ_OK : PCBZ_EDEVICE;
}

int pcbz_gemm_bf16(int M, int N, int K, const uint16_t *d_a, const uint16_t *d_b, float *d_c, void *stream) {
  if (M <= 0 || N <= 0 || K <= 0 || !d_a || !d_b || !d_c) return PCBZ_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  gemm_bf16(M, N, K, d_a, K, 1, d_b, N, 1, d_c, N, 1, nullptr, s);
  return hipStreamSynchronize(s) == hipSuccess ? PCBZ_OK : PCBZ_EDEVICE;
}

}  // extern "C"
