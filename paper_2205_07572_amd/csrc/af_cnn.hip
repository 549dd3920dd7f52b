// af_cnn.hip -- learned regrid tagger on gfx950 (a project addition, not part
// of the paper's method).
//
// Network: three 3x3 convolutions (zero "same" padding, 16x16 inputs,
// nin -> 32 -> 32 -> 32 channels, ReLU), global average pooling, linear head
// 32 -> 3 (coarsen / keep / refine), softmax cross-entropy.  Parameters are
// FP32 masters packed as W1[co][ci][3][3], b1, W2, b2, W3, b3, Wh[3][32], bh.
//
// The convolutions run as implicit GEMMs on the matrix cores: im2col gathers
// (BF16), one strided GEMM kernel built on v_mfma_f32_16x16x32_bf16 (BF16
// operands, FP32 accumulation) for forward, input-gradient and
// weight-gradient products, col2im sums.  Bias, ReLU, pooling, head, loss
// and the Adam update are FP32 elementwise kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "af.h"
#include "af_internal.h"

namespace af {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kImg = 16, kPix = 256, kWidth = 32, kClasses = 3;

// FP32 -> BF16, round to nearest even (NaN and Inf pass through).
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return uint16_t(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }

// ---------------------------------------------------------------------------
// C(i,j) (+)= sum_k A(i,k) B(j,k), A and B BF16 with arbitrary strides, C FP32.
// One wavefront computes a 16x16 tile: lane l loads A row i0 + l%16 and
// B row j0 + l%16 at k = k0 + 8 (l/16) + e, e < 8 (the same k order for both
// operands, so the hardware's internal k order does not matter), and the
// accumulator holds C rows i0 + 4 (l/16) + r, r < 4, column j0 + l%16.
// blockIdx.z splits K into chunks (multiples of 32); chunk z writes its
// partial product to part[z][i][j] and k_sum_chunks adds the chunks in
// order, so the result does not depend on scheduling.
// A lane's 8 values of one operand are one 16-byte load where they are
// contiguous and aligned (unit k stride, row stride a multiple of 8, K a
// multiple of 8, so that a group of 8 lies wholly inside or outside
// [0, K)); else 8 element loads.  With X set, A is the im2col matrix of the
// BF16 NHWC images X (cp channels, cp a multiple of 8), read in place: the
// 8 values of a lane are 8 channels of one pixel of one tap, zero outside
// the image.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const uint16_t* A;
  long sai, sak;
  const uint16_t* B;
  long sbj, sbk;
  float* C;
  long sci, scj;
  int M, N, K, kchunk;
  float* part;  // [nz][M][N] when K is split, else null
  const uint16_t* X = nullptr;  // implicit im2col source (then A is unused)
  int cp = 0;
  int avec = 0, bvec = 0;       // set by gemm(): 16-byte loads for A, B
};

__global__ __launch_bounds__(256) void k_gemm_bf16(const GemmArgs g) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_n = (g.N + 15) >> 4;
  const int tile = blockIdx.x * 4 + wave;
  const int ti = tile / tiles_n, tj = tile - ti * tiles_n;
  if (ti * 16 >= g.M) return;  // uniform per wavefront
  const int i = ti * 16 + (lane & 15), j = tj * 16 + (lane & 15);
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  const u16x8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    u16x8 a, b;
    const int ks = k0 + 8 * (lane >> 4);  // this lane's first k
    if (g.X) {
      a = zero8;
      if (ks < ke && i < g.M) {
        const int tap = ks / g.cp, ci = ks - tap * g.cp;
        const int bi = i / kPix, p = i - bi * kPix;
        const int y = p / kImg + tap / 3 - 1, x = p % kImg + tap % 3 - 1;
        if (y >= 0 && y < kImg && x >= 0 && x < kImg)
          a = *reinterpret_cast<const u16x8*>(g.X + (long(bi) * kPix + y * kImg + x) * g.cp + ci);
      }
    } else if (g.avec) {
      a = (ks < ke && i < g.M) ? *reinterpret_cast<const u16x8*>(g.A + i * g.sai + ks) : zero8;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = ks + e;
        a[e] = (k < ke && i < g.M) ? g.A[i * g.sai + k * g.sak] : uint16_t(0);
      }
    }
    if (g.bvec) {
      b = (ks < ke && j < g.N) ? *reinterpret_cast<const u16x8*>(g.B + j * g.sbj + ks) : zero8;
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = ks + e;
        b[e] = (k < ke && j < g.N) ? g.B[j * g.sbj + k * g.sbk] : uint16_t(0);
      }
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                  acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = ti * 16 + 4 * (lane >> 4) + r, col = tj * 16 + (lane & 15);
    if (row < g.M && col < g.N) {
      if (g.part) g.part[(size_t(blockIdx.z) * g.M + row) * g.N + col] = acc[r];
      else g.C[row * g.sci + col * g.scj] = acc[r];
    }
  }
}

// C(i, j) = sum over z = 0, 1, ... of part[z][i][j], in that order.
__global__ void k_sum_chunks(const float* part, int nz, int M, int N, float* C, long sci, long scj) {
  const long n = long(M) * N;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < n; e += long(gridDim.x) * blockDim.x) {
    float s = part[e];
    for (int z = 1; z < nz; ++z) s += part[size_t(z) * n + e];
    const long i = e / N, j = e - i * N;
    C[i * sci + j * scj] = s;
  }
}

// Chunks a split GEMM of this K uses: about K / 4096, at most kMaxChunks.
constexpr int kMaxChunks = 64;
int gemm_chunks(long K, int ksplit) {
  const long kc = ((K + ksplit - 1) / ksplit + 31) / 32 * 32;
  return int((K + kc - 1) / kc);
}

// ws: workspace of at least nz * M * N floats when ksplit > 1.
static hipError_t gemm(const GemmArgs& g0, int ksplit, float* ws, hipStream_t st) {
  GemmArgs g = g0;
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  g.avec = !g.X && g.sak == 1 && g.sai % 8 == 0 && g.K % 8 == 0 && al16(g.A);
  g.bvec = g.sbk == 1 && g.sbj % 8 == 0 && g.K % 8 == 0 && al16(g.B);
  if (g.X && (g.cp % 8 != 0 || g.K != 9 * g.cp || !al16(g.X))) return hipErrorInvalidValue;
  const int tiles = ((g.M + 15) / 16) * ((g.N + 15) / 16);
  const int kc = ((g.K + ksplit - 1) / ksplit + 31) / 32 * 32;
  g.kchunk = kc;
  const int nz = (g.K + kc - 1) / kc;
  g.part = nz > 1 ? ws : nullptr;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(unsigned((tiles + 3) / 4), 1, unsigned(nz)), dim3(256), 0, st, g);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || nz == 1) return e;
  const long n = long(g.M) * g.N;
  hipLaunchKernelGGL(k_sum_chunks, dim3(unsigned(std::min<long>((n + 255) / 256, 4096))), dim3(256), 0, st, ws, nz,
                     g.M, g.N, g.C, g.sci, g.scj);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// im2col: Xcol[m = b*256 + y*16 + x][k = tap*cp + ci] = X(b, y+ky-1, x+kx-1, ci)
// (zero outside the image and for ci >= c).  Source either FP32 NCHW (the
// API input, rounded to BF16 here) or BF16 NHWC with cp channels.
// ---------------------------------------------------------------------------
__global__ void k_im2col(const float* xf, const uint16_t* xb, int B, int c, int cp, uint16_t* col) {
  const long K = 9L * cp;
  const long total = long(B) * kPix * K;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < total; e += long(gridDim.x) * blockDim.x) {
    const long m = e / K;
    const int k = int(e - m * K);
    const int tap = k / cp, ci = k - tap * cp;
    const int b = int(m / kPix), p = int(m - long(b) * kPix);
    const int y = p / kImg + tap / 3 - 1, x = p % kImg + tap % 3 - 1;
    uint16_t v = 0;
    if (ci < c && y >= 0 && y < kImg && x >= 0 && x < kImg) {
      if (xf) v = f2bf(xf[(long(b) * c + ci) * kPix + y * kImg + x]);
      else v = xb[(long(b) * kPix + y * kImg + x) * cp + ci];
    }
    col[e] = v;
  }
}

// X(b, c, y, x) FP32 NCHW -> BF16 NHWC with cp >= c channels (zero-padded)
__global__ void k_to_nhwc(const float* xf, int B, int c, int cp, uint16_t* xb) {
  const long total = long(B) * kPix * cp;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < total; e += long(gridDim.x) * blockDim.x) {
    const int ci = int(e % cp);
    const long bp = e / cp;
    const int b = int(bp / kPix), p = int(bp - long(b) * kPix);
    xb[e] = ci < c ? f2bf(xf[(long(b) * c + ci) * kPix + p]) : uint16_t(0);
  }
}

// dX(b, y, x, ci) = sum over taps of dXcol[b, (y-ky+1, x-kx+1)][tap*cp + ci]
__global__ void k_col2im(const float* dcol, int B, int cp, float* dx) {
  const long total = long(B) * kPix * cp;
  const long K = 9L * cp;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < total; e += long(gridDim.x) * blockDim.x) {
    const int ci = int(e % cp);
    const long bp = e / cp;
    const int b = int(bp / kPix), p = int(bp - long(b) * kPix);
    const int y = p / kImg, x = p % kImg;
    float s = 0.f;
    for (int tap = 0; tap < 9; ++tap) {
      const int yy = y - tap / 3 + 1, xx = x - tap % 3 + 1;
      if (yy < 0 || yy >= kImg || xx < 0 || xx >= kImg) continue;
      s += dcol[(long(b) * kPix + yy * kImg + xx) * K + tap * cp + ci];
    }
    dx[e] = s;
  }
}

// Z = Y + bias (FP32 [M][32]); A = relu(Z) stored BF16 (next layer input)
// and FP32 (pooling of the last layer).
__global__ void k_bias_relu(float* z, const float* bias, long M, uint16_t* ab, float* af32) {
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < M * kWidth; e += long(gridDim.x) * blockDim.x) {
    const float v = z[e] + bias[e % kWidth];
    z[e] = v;
    const float a = v > 0.f ? v : 0.f;
    ab[e] = f2bf(a);
    if (af32) af32[e] = a;
  }
}

// Weight matrices from the FP32 masters: Wm[co][tap*cp + ci] (forward) and
// Wt[tap*cp + ci][co] (input gradient), BF16; zero for padded ci.
__global__ void k_pack_weights(const float* W, int c, int cp, uint16_t* Wm, uint16_t* Wt) {
  const int K = 9 * cp;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < kWidth * K; e += gridDim.x * blockDim.x) {
    const int co = e / K, k = e - co * K, tap = k / cp, ci = k - tap * cp;
    const uint16_t v = ci < c ? f2bf(W[((co * c + ci) * 3 + tap / 3) * 3 + tap % 3]) : uint16_t(0);
    Wm[e] = v;
    Wt[k * kWidth + co] = v;
  }
}

// Head: pooled mean, logits, and (if labels) softmax cross-entropy, its
// gradient w.r.t. the head parameters and the broadcast pooling gradient.
// One block of 32 x 8 threads per 8 samples.  Sample b writes its terms of
// the batch sums to hp[b][kHeadTerms] (loss, Wh [3][32], bh [3]);
// k_head_sum adds them in sample order.
constexpr int kHeadTerms = 1 + kClasses * kWidth + kClasses;
__global__ void k_head(const float* a3, int B, const float* Wh, const float* bh, float* logits, const int32_t* labels,
                       float* hp, float* dA3) {
  const int c = threadIdx.x & 31, sb = threadIdx.x >> 5;
  const int b = blockIdx.x * 8 + sb;
  __shared__ float pooled[8][kWidth], lg[8][4];
  if (b < B) {
    float s = 0.f;
    for (int p = 0; p < kPix; ++p) s += a3[(long(b) * kPix + p) * kWidth + c];
    pooled[sb][c] = s * (1.0f / kPix);
  }
  __syncthreads();
  if (b < B && c < kClasses) {
    float s = bh[c];
    for (int k = 0; k < kWidth; ++k) s += Wh[c * kWidth + k] * pooled[sb][k];
    lg[sb][c] = s;
    logits[b * kClasses + c] = s;
  }
  __syncthreads();
  if (!labels || b >= B) return;
  const int lab = min(max(int(labels[b]), 0), kClasses - 1);
  const float mx = fmaxf(lg[sb][0], fmaxf(lg[sb][1], lg[sb][2]));
  float den = 0.f;
  for (int k = 0; k < kClasses; ++k) den += expf(lg[sb][k] - mx);
  float dl[kClasses];
  for (int k = 0; k < kClasses; ++k) dl[k] = (expf(lg[sb][k] - mx) / den - (k == lab ? 1.f : 0.f)) / B;
  float* const t = hp + size_t(b) * kHeadTerms;
  if (c == 0) t[0] = -(lg[sb][lab] - mx - logf(den)) / B;
  float dp = 0.f;
  for (int k = 0; k < kClasses; ++k) {
    t[1 + k * kWidth + c] = dl[k] * pooled[sb][c];
    dp += dl[k] * Wh[k * kWidth + c];
  }
  if (c < kClasses) t[1 + kClasses * kWidth + c] = dl[c];
  for (int p = 0; p < kPix; ++p) dA3[(long(b) * kPix + p) * kWidth + c] = dp * (1.0f / kPix);
}

// loss, gWh, gbh: the per-sample terms summed over b = 0, 1, ... in order.
__global__ void k_head_sum(const float* hp, int B, float* loss, float* gWh, float* gbh) {
  const int e = threadIdx.x;
  if (e >= kHeadTerms) return;
  float s = 0.f;
  for (int b = 0; b < B; ++b) s += hp[size_t(b) * kHeadTerms + e];
  if (e == 0) *loss = s;
  else if (e <= kClasses * kWidth) gWh[e - 1] = s;
  else gbh[e - 1 - kClasses * kWidth] = s;
}

// G = dA * relu'(Z): FP32 for the bias gradient, BF16 for the products.
// Block k writes its bias partial sums to bpart[k][32] (a thread's elements
// all belong to channel threadIdx.x % 32, since the stride is a multiple of
// 32); k_bias_sum adds the blocks in order.
__global__ void k_relu_back(const float* dA, const float* z, long M, uint16_t* gb, float* bpart) {
  __shared__ float part[256];
  const int c = threadIdx.x & 31;
  float s = 0.f;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < M * kWidth; e += long(gridDim.x) * blockDim.x) {
    const float g = z[e] > 0.f ? dA[e] : 0.f;
    gb[e] = f2bf(g);
    s += g;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x < 32) {
    float t = 0.f;
    for (int w = 0; w < 8; ++w) t += part[w * 32 + c];
    bpart[size_t(blockIdx.x) * kWidth + c] = t;
  }
}

__global__ void k_bias_sum(const float* bpart, int nblocks, float* gbias) {
  const int c = threadIdx.x;
  if (c >= kWidth) return;
  float s = 0.f;
  for (int k = 0; k < nblocks; ++k) s += bpart[size_t(k) * kWidth + c];
  gbias[c] = s;
}

// dW packed order from the GEMM layout dWm[co][tap*cp + ci].
__global__ void k_unpack_wgrad(const float* dWm, int c, int cp, float* gW) {
  const int n = kWidth * c * 9;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const int co = e / (c * 9), r = e - co * c * 9, ci = r / 9, tap = r - ci * 9;
    gW[e] = dWm[co * 9 * cp + tap * cp + ci];
  }
}

__global__ void k_adam(float* p, float* m1, float* m2, const float* g, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
    const float gi = g[e];
    const float a = b1 * m1[e] + (1.f - b1) * gi;
    const float v = b2 * m2[e] + (1.f - b2) * gi * gi;
    m1[e] = a;
    m2[e] = v;
    p[e] -= lr * (a / c1) / (sqrtf(v / c2) + eps);
  }
}

// Features of leaves (m = 16): 12 channels (p,u,v) x (avg, corner, xedge,
// yedge) of the owned DOFs of every interior cell, and one channel with the
// leaf level; each standardised with (x - mean[c]) * inv_std[c].
template <typename T>
struct DofPtrs {
  const T* p[2][4];
};

template <typename T>
__global__ void k_features(const DofPtrs<T> D, uint32_t mask, int npatch, int pitch, int ncomp,
                           const int32_t* plevel, int first, int n, const float* mean, const float* inv_std, int nin,
                           float* x) {
  const long total = long(n) * nin * kPix;
  for (long e = blockIdx.x * long(blockDim.x) + threadIdx.x; e < total; e += long(gridDim.x) * blockDim.x) {
    const int p = int(e % kPix);
    const long bc = e / kPix;
    const int ch = int(bc % nin), b = int(bc / nin);
    const int leaf = first + b;
    const int l = plevel[leaf];
    float v;
    if (ch >= 12 || ch / 4 >= ncomp) {
      v = ch >= 12 ? float(l) : 0.f;
    } else {
      const int q = ch / 4, kind = ch % 4;
      const T* base = D.p[(mask >> l) & 1][kind];
      const int i = p % kImg, j = p / kImg;
      v = float(base[((size_t(q) * npatch + leaf) * (kImg + 5) + (j + kGhost)) * pitch + (i + kGhost)]);
    }
    x[e] = (v - mean[ch]) * inv_std[ch];
  }
}

// Learned tags with the plain criterion as fallback: refine if either says
// refine; coarsen only if both say coarsen; a non-finite output uses the
// plain tag.  Level limits as for the plain tagger.
__global__ void k_combine_tags(const float* logits, const int8_t* plain, const int32_t* plevel, int first, int n,
                               int lmax, int8_t* out, int8_t* learned) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const float* L = logits + b * kClasses;
  const int leaf = first + b;
  const int8_t pt = plain[leaf];
  int8_t t;
  if (!isfinite(L[0]) || !isfinite(L[1]) || !isfinite(L[2])) {
    t = pt;
    if (learned) learned[leaf] = 2;  // marks a fallback
  } else {
    const int cls = (L[2] > L[1] && L[2] > L[0]) ? 2 : (L[0] > L[1] ? 0 : 1);
    const int8_t lt = int8_t(cls - 1);
    if (learned) learned[leaf] = lt;
    if (lt == 1 || pt == 1) t = 1;
    else if (lt == -1 && pt == -1) t = -1;
    else t = 0;
  }
  const int l = plevel[leaf];
  if (t == 1 && l >= lmax) t = 0;
  if (t == -1 && l == 0) t = 0;
  out[leaf] = t;
}

}  // namespace af

// ===========================================================================
// Host side
// ===========================================================================
using namespace af;

struct af_cnn {
  int nin, cp1, nparams;
  size_t off_w[3], off_b[3], off_wh, off_bh;
  float* d_params = nullptr;  // FP32 masters
  float* d_m1 = nullptr;
  float* d_m2 = nullptr;
  float* d_grad = nullptr;
  // packed BF16 weights
  uint16_t* d_wm[3] = {nullptr, nullptr, nullptr};
  uint16_t* d_wt[3] = {nullptr, nullptr, nullptr};
  // activation workspace for a batch of up to cap samples
  int cap = 0;
  uint16_t* d_col[3] = {nullptr, nullptr, nullptr};
  float* d_z[3] = {nullptr, nullptr, nullptr};
  uint16_t* d_ab[3] = {nullptr, nullptr, nullptr};
  float* d_a3 = nullptr;
  float* d_dA = nullptr;
  float* d_dcol = nullptr;
  uint16_t* d_g = nullptr;
  float* d_dwm = nullptr;
  float* d_logits = nullptr;
  float* d_feat = nullptr;
  float* d_part = nullptr;  // split-K, bias and head partial sums (fixed-order reductions)
  float* d_norm = nullptr;  // mean[nin], inv_std[nin]
  std::string err;
};

namespace {
thread_local std::string g_cnn_err;
af_status cfail(af_status s, const std::string& m) {
  g_cnn_err = m;
  return s;
}
#define CNN_HIP(call)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (call);                                                                             \
    if (e_ != hipSuccess) return cfail(AF_ERR_DEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

int grid_for(long n) { return int(std::min<long>((n + 255) / 256, 8192)); }
// K split of the weight-gradient GEMMs (K = B * 256 pixels): chunks of about
// 4096 pixels, at most kMaxChunks
int wgrad_split(long M) { return int(std::min<long>(std::max<long>(1, M / 4096), kMaxChunks)); }

af_status ensure_batch(af_cnn* c, int B) {
  if (B <= c->cap) return AF_OK;
  for (int l = 0; l < 3; ++l) {
    (void)hipFree(c->d_col[l]);
    (void)hipFree(c->d_z[l]);
    (void)hipFree(c->d_ab[l]);
  }
  (void)hipFree(c->d_a3);
  (void)hipFree(c->d_dA);
  (void)hipFree(c->d_dcol);
  (void)hipFree(c->d_g);
  (void)hipFree(c->d_logits);
  (void)hipFree(c->d_feat);
  (void)hipFree(c->d_part);
  const long M = long(B) * kPix;
  for (int l = 0; l < 3; ++l) {
    const int cp = l == 0 ? c->cp1 : kWidth;
    CNN_HIP(hipMalloc(&c->d_col[l], size_t(M) * 9 * cp * 2));
    CNN_HIP(hipMalloc(&c->d_z[l], size_t(M) * kWidth * 4));
    CNN_HIP(hipMalloc(&c->d_ab[l], size_t(M) * kWidth * 2));
  }
  CNN_HIP(hipMalloc(&c->d_a3, size_t(M) * kWidth * 4));
  CNN_HIP(hipMalloc(&c->d_dA, size_t(M) * kWidth * 4));
  CNN_HIP(hipMalloc(&c->d_dcol, size_t(M) * 9 * kWidth * 4));
  CNN_HIP(hipMalloc(&c->d_g, size_t(M) * kWidth * 2));
  CNN_HIP(hipMalloc(&c->d_logits, size_t(B) * kClasses * 4));
  CNN_HIP(hipMalloc(&c->d_feat, size_t(B) * c->nin * kPix * 4));
  // partial sums: split-K chunks of the weight-gradient GEMMs, per-block
  // bias sums, per-sample head terms
  const size_t part = std::max({size_t(gemm_chunks(M, wgrad_split(M))) * kWidth * 9 * kWidth,
                                size_t(grid_for(M * kWidth)) * kWidth, size_t(B) * kHeadTerms});
  CNN_HIP(hipMalloc(&c->d_part, part * 4));
  c->cap = B;
  return AF_OK;
}

af_status pack_weights(af_cnn* c, hipStream_t st) {
  for (int l = 0; l < 3; ++l) {
    const int cin = l == 0 ? c->nin : kWidth, cp = l == 0 ? c->cp1 : kWidth;
    hipLaunchKernelGGL(k_pack_weights, dim3(grid_for(kWidth * 9 * cp)), dim3(256), 0, st, c->d_params + c->off_w[l],
                       cin, cp, c->d_wm[l], c->d_wt[l]);
    CNN_HIP(hipGetLastError());
  }
  return AF_OK;
}

// With cols (training), each layer's im2col matrix is written to d_col[l]
// (the weight gradient reads it); without (inference), the input is
// converted once to BF16 NHWC and every layer's GEMM reads its im2col
// matrix in place from the NHWC images.  Both give the same products in the
// same k order, bit for bit.
af_status forward(af_cnn* c, const float* x, int B, hipStream_t st, bool cols = true) {
  af_status s = ensure_batch(c, B);
  if (s != AF_OK) return s;
  if ((s = pack_weights(c, st)) != AF_OK) return s;
  const long M = long(B) * kPix;
  if (!cols) {
    // layer-0 input as BF16 NHWC with cp1 channels (d_col[0] holds 9x that)
    hipLaunchKernelGGL(k_to_nhwc, dim3(grid_for(M * c->cp1)), dim3(256), 0, st, x, B, c->nin, c->cp1, c->d_col[0]);
    CNN_HIP(hipGetLastError());
  }
  for (int l = 0; l < 3; ++l) {
    const int cp = l == 0 ? c->cp1 : kWidth;
    const int K = 9 * cp;
    GemmArgs g{c->d_col[l], K, 1, c->d_wm[l], K, 1, c->d_z[l], kWidth, 1, int(M), kWidth, K, 0, nullptr};
    if (cols) {
      hipLaunchKernelGGL(k_im2col, dim3(grid_for(M * K)), dim3(256), 0, st, l == 0 ? x : nullptr,
                         l == 0 ? nullptr : c->d_ab[l - 1], B, l == 0 ? c->nin : kWidth, cp, c->d_col[l]);
      CNN_HIP(hipGetLastError());
    } else {
      g.X = l == 0 ? c->d_col[0] : c->d_ab[l - 1];
      g.cp = cp;
    }
    CNN_HIP(gemm(g, 1, nullptr, st));
    hipLaunchKernelGGL(k_bias_relu, dim3(grid_for(M * kWidth)), dim3(256), 0, st, c->d_z[l],
                       c->d_params + c->off_b[l], M, c->d_ab[l], l == 2 ? c->d_a3 : nullptr);
    CNN_HIP(hipGetLastError());
  }
  return AF_OK;
}

}  // namespace

extern "C" {

const char* af_cnn_last_error(void) { return g_cnn_err.c_str(); }

af_status af_cnn_create(int32_t nin, af_cnn** out) {
  if (!out || nin < 1 || nin > 32) return cfail(AF_ERR_ARG, "nin must be in [1, 32]");
  auto c = std::make_unique<af_cnn>();
  c->nin = nin;
  c->cp1 = (nin + 7) / 8 * 8;
  size_t o = 0;
  for (int l = 0; l < 3; ++l) {
    const int cin = l == 0 ? nin : kWidth;
    c->off_w[l] = o;
    o += size_t(kWidth) * cin * 9;
    c->off_b[l] = o;
    o += kWidth;
  }
  c->off_wh = o;
  o += kClasses * kWidth;
  c->off_bh = o;
  o += kClasses;
  c->nparams = int(o);
  CNN_HIP(hipMalloc(&c->d_params, o * 4));
  CNN_HIP(hipMalloc(&c->d_m1, o * 4));
  CNN_HIP(hipMalloc(&c->d_m2, o * 4));
  CNN_HIP(hipMalloc(&c->d_grad, o * 4));
  CNN_HIP(hipMemset(c->d_params, 0, o * 4));
  CNN_HIP(hipMemset(c->d_m1, 0, o * 4));
  CNN_HIP(hipMemset(c->d_m2, 0, o * 4));
  for (int l = 0; l < 3; ++l) {
    const int cp = l == 0 ? c->cp1 : kWidth;
    CNN_HIP(hipMalloc(&c->d_wm[l], size_t(kWidth) * 9 * cp * 2));
    CNN_HIP(hipMalloc(&c->d_wt[l], size_t(kWidth) * 9 * cp * 2));
  }
  CNN_HIP(hipMalloc(&c->d_dwm, size_t(kWidth) * 9 * kWidth * 4));
  CNN_HIP(hipMalloc(&c->d_norm, size_t(2) * nin * 4));
  std::vector<float> norm(2 * nin, 0.f);
  for (int i = 0; i < nin; ++i) norm[nin + i] = 1.f;
  CNN_HIP(hipMemcpy(c->d_norm, norm.data(), norm.size() * 4, hipMemcpyHostToDevice));
  *out = c.release();
  return AF_OK;
}

af_status af_cnn_destroy(af_cnn* c) {
  if (!c) return AF_OK;
  (void)hipFree(c->d_params);
  (void)hipFree(c->d_m1);
  (void)hipFree(c->d_m2);
  (void)hipFree(c->d_grad);
  for (int l = 0; l < 3; ++l) {
    (void)hipFree(c->d_wm[l]);
    (void)hipFree(c->d_wt[l]);
    (void)hipFree(c->d_col[l]);
    (void)hipFree(c->d_z[l]);
    (void)hipFree(c->d_ab[l]);
  }
  (void)hipFree(c->d_a3);
  (void)hipFree(c->d_dA);
  (void)hipFree(c->d_dcol);
  (void)hipFree(c->d_g);
  (void)hipFree(c->d_dwm);
  (void)hipFree(c->d_logits);
  (void)hipFree(c->d_feat);
  (void)hipFree(c->d_part);
  (void)hipFree(c->d_norm);
  delete c;
  return AF_OK;
}

int32_t af_cnn_num_params(const af_cnn* c) { return c ? c->nparams : -1; }

af_status af_cnn_set_params(af_cnn* c, const float* host) {
  if (!c || !host) return cfail(AF_ERR_ARG, "null argument");
  CNN_HIP(hipMemcpy(c->d_params, host, size_t(c->nparams) * 4, hipMemcpyHostToDevice));
  CNN_HIP(hipMemset(c->d_m1, 0, size_t(c->nparams) * 4));
  CNN_HIP(hipMemset(c->d_m2, 0, size_t(c->nparams) * 4));
  return AF_OK;
}

af_status af_cnn_get_params(const af_cnn* c, float* host) {
  if (!c || !host) return cfail(AF_ERR_ARG, "null argument");
  CNN_HIP(hipMemcpy(host, c->d_params, size_t(c->nparams) * 4, hipMemcpyDeviceToHost));
  return AF_OK;
}

af_status af_cnn_set_normalization(af_cnn* c, const float* mean, const float* inv_std) {
  if (!c || !mean || !inv_std) return cfail(AF_ERR_ARG, "null argument");
  std::vector<float> v(mean, mean + c->nin);
  v.insert(v.end(), inv_std, inv_std + c->nin);
  CNN_HIP(hipMemcpy(c->d_norm, v.data(), v.size() * 4, hipMemcpyHostToDevice));
  return AF_OK;
}

af_status af_cnn_forward(af_cnn* c, const float* x, int32_t B, float* logits, float* acts, hipStream_t st) {
  if (!c || !x || !logits || B <= 0) return cfail(AF_ERR_ARG, "bad argument");
  af_status s = forward(c, x, B, st, false);
  if (s != AF_OK) return s;
  hipLaunchKernelGGL(k_head, dim3((B + 7) / 8), dim3(256), 0, st, c->d_a3, B, c->d_params + c->off_wh,
                     c->d_params + c->off_bh, logits, nullptr, nullptr, nullptr);
  CNN_HIP(hipGetLastError());
  if (acts) {
    // pre-activations of the three layers, FP32 [3][B*256][32] (NHWC)
    const size_t M = size_t(B) * kPix;
    for (int l = 0; l < 3; ++l)
      CNN_HIP(hipMemcpyAsync(acts + l * M * kWidth, c->d_z[l], M * kWidth * 4, hipMemcpyDeviceToDevice, st));
  }
  return AF_OK;
}

af_status af_cnn_loss_grad(af_cnn* c, const float* x, const int32_t* labels, int32_t B, float* loss, float* grad,
                           float* dacts, hipStream_t st) {
  if (!c || !x || !labels || !loss || B <= 0) return cfail(AF_ERR_ARG, "bad argument");
  float* G = grad ? grad : c->d_grad;
  af_status s = forward(c, x, B, st);
  if (s != AF_OK) return s;
  const long M = long(B) * kPix;
  // every entry of G and loss is written below (no accumulation across calls)
  hipLaunchKernelGGL(k_head, dim3((B + 7) / 8), dim3(256), 0, st, c->d_a3, B, c->d_params + c->off_wh,
                     c->d_params + c->off_bh, c->d_logits, labels, c->d_part, c->d_dA);
  CNN_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_head_sum, dim3(1), dim3(128), 0, st, c->d_part, B, loss, G + c->off_wh, G + c->off_bh);
  CNN_HIP(hipGetLastError());
  for (int l = 2; l >= 0; --l) {
    const int cin = l == 0 ? c->nin : kWidth, cp = l == 0 ? c->cp1 : kWidth;
    const int K = 9 * cp;
    if (dacts)  // the upstream gradient this layer's backward consumes
      CNN_HIP(hipMemcpyAsync(dacts + size_t(l) * M * kWidth, c->d_dA, size_t(M) * kWidth * 4, hipMemcpyDeviceToDevice,
                             st));
    const int nb = grid_for(M * kWidth);
    hipLaunchKernelGGL(k_relu_back, dim3(nb), dim3(256), 0, st, c->d_dA, c->d_z[l], M, c->d_g, c->d_part);
    CNN_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_bias_sum, dim3(1), dim3(64), 0, st, c->d_part, nb, G + c->off_b[l]);
    CNN_HIP(hipGetLastError());
    // dWm[co][k] = sum_m G[m][co] Xcol[m][k]
    GemmArgs gw{c->d_g, 1, kWidth, c->d_col[l], 1, K, c->d_dwm, K, 1, kWidth, K, int(M), 0, nullptr};
    CNN_HIP(gemm(gw, wgrad_split(M), c->d_part, st));
    hipLaunchKernelGGL(k_unpack_wgrad, dim3(grid_for(kWidth * cin * 9)), dim3(256), 0, st, c->d_dwm, cin, cp,
                       G + c->off_w[l]);
    CNN_HIP(hipGetLastError());
    if (l > 0) {
      // dXcol[m][k] = sum_co G[m][co] Wm[co][k]
      GemmArgs gx{c->d_g, kWidth, 1, c->d_wt[l], kWidth, 1, c->d_dcol, K, 1, int(M), K, kWidth, 0, nullptr};
      CNN_HIP(gemm(gx, 1, nullptr, st));
      hipLaunchKernelGGL(k_col2im, dim3(grid_for(M * cp)), dim3(256), 0, st, c->d_dcol, B, cp, c->d_dA);
      CNN_HIP(hipGetLastError());
    }
  }
  return AF_OK;
}

af_status af_cnn_adam_step(af_cnn* c, const float* grad, float lr, int32_t t, hipStream_t st) {
  if (!c || t < 1) return cfail(AF_ERR_ARG, "bad argument");
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, float(t)), c2 = 1.f - std::pow(b2, float(t));
  hipLaunchKernelGGL(k_adam, dim3(grid_for(c->nparams)), dim3(256), 0, st, c->d_params, c->d_m1, c->d_m2,
                     grad ? grad : c->d_grad, c->nparams, lr, b1, b2, 1e-8f, c1, c2);
  CNN_HIP(hipGetLastError());
  return AF_OK;
}

}  // extern "C"

// Feature extraction and learned tagging need the AF context and hierarchy;
// they are implemented with the accessors below (defined in af_api.cpp).
struct AfTagView {
  bool fp32;
  int ncomp, m, npatch, pitch, lmax, nleaves;
  const void* dof0[4];
  const void* dof1[4];
  const int32_t* plevel;
};
extern "C" af_status af_internal_tag_view(const af_ctx* ctx, const af_hier* h, const af_state* bufs, AfTagView* v);

extern "C" {

af_status af_cnn_features(af_ctx* ctx, af_cnn* c, const af_hier* h, const af_state* bufs, uint32_t mask,
                          float* x, hipStream_t st) {
  if (!ctx || !c || !h || !x) return cfail(AF_ERR_ARG, "null argument");
  AfTagView v;
  af_status s = af_internal_tag_view(ctx, h, bufs, &v);
  if (s != AF_OK) return cfail(s, "af_cnn_features: bad context, hierarchy or buffers");
  if (v.m != kImg) return cfail(AF_ERR_ARG, "af_cnn_features: the tagger takes 16x16 patches");
  const long total = long(v.nleaves) * c->nin * kPix;
  if (v.fp32) {
    DofPtrs<float> D;
    for (int k = 0; k < 4; ++k) {
      D.p[0][k] = static_cast<const float*>(v.dof0[k]);
      D.p[1][k] = static_cast<const float*>(v.dof1[k]);
    }
    hipLaunchKernelGGL(k_features<float>, dim3(grid_for(total)), dim3(256), 0, st, D, mask, v.npatch, v.pitch,
                       v.ncomp, v.plevel, 0, v.nleaves, c->d_norm, c->d_norm + c->nin, c->nin, x);
  } else {
    DofPtrs<double> D;
    for (int k = 0; k < 4; ++k) {
      D.p[0][k] = static_cast<const double*>(v.dof0[k]);
      D.p[1][k] = static_cast<const double*>(v.dof1[k]);
    }
    hipLaunchKernelGGL(k_features<double>, dim3(grid_for(total)), dim3(256), 0, st, D, mask, v.npatch, v.pitch,
                       v.ncomp, v.plevel, 0, v.nleaves, c->d_norm, c->d_norm + c->nin, c->nin, x);
  }
  CNN_HIP(hipGetLastError());
  return AF_OK;
}

af_status af_cnn_tag(af_ctx* ctx, af_cnn* c, const af_hier* h, const af_state* bufs, uint32_t mask,
                     const int8_t* plain, int8_t* tags, int8_t* learned, hipStream_t st) {
  if (!ctx || !c || !h || !plain || !tags) return cfail(AF_ERR_ARG, "null argument");
  AfTagView v;
  af_status s = af_internal_tag_view(ctx, h, bufs, &v);
  if (s != AF_OK) return cfail(s, "af_cnn_tag: bad context, hierarchy or buffers");
  if ((s = ensure_batch(c, v.nleaves)) != AF_OK) return s;
  if ((s = af_cnn_features(ctx, c, h, bufs, mask, c->d_feat, st)) != AF_OK) return s;
  if ((s = af_cnn_forward(c, c->d_feat, v.nleaves, c->d_logits, nullptr, st)) != AF_OK) return s;
  hipLaunchKernelGGL(k_combine_tags, dim3((v.nleaves + 255) / 256), dim3(256), 0, st, c->d_logits, plain, v.plevel,
                     0, v.nleaves, v.lmax, tags, learned);
  CNN_HIP(hipGetLastError());
  return AF_OK;
}

}  // extern "C"
