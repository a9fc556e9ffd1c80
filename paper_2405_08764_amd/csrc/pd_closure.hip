// Learned closure kernels: the network that stands in for a patch's micro-burst (not in
// the paper; the patch scheme produces its training targets and stays its fallback).
//
// Inputs of patch p at macro node (i, j): the 5x5 macro stencil (indices wrap on a
// periodic axis, clamp otherwise), the coefficient rates at the patch centre and the micro
// cell Peclet numbers (which carry the scale factors and the micro spacing).  The network predicts a correction to the macro finite-difference
// operator F0 at the node, scaled by s = kappa sigma + 1e-3 (|g| + |phi U|):
// F_hat = F0 + s y_hat, then U_np1 = U + dt_macro F_hat (eq. Extrapolation).
//
// Training (FP32 master weights): tiled FP32 GEMMs, fused bias + GELU, its derivative,
// mean-squared-error head, Adam.  Inference: bfloat16 MFMA (32x32x8, FP32 accumulation)
// for the two hidden layers, FP32 for the output dot product.
#include "pd_internal.h"

namespace pdk {
namespace {

// ------------------------------------------------------------------------- features

struct Feat {
  float x[CL_FEAT];
  double F0, s, u;
  int node;
};

__device__ __forceinline__ void closure_features(const Geo& g, const SrcInfo& src,
                                                 const double* st, const double* U,
                                                 double t_n, Feat& f) {
  const int i = (int)st[0], j = (int)st[1];
  const int nx = g.n_xi, ne = g.n_eta;
  double S[5][5];
#pragma unroll
  for (int b = 0; b < 5; ++b) {
    int jj = j + b - 2;
    jj = jj < 0 ? 0 : (jj > ne - 1 ? ne - 1 : jj);
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      int ii = i + a - 2;
      if (g.periodic) ii = (ii + nx) % nx;
      else ii = ii < 0 ? 0 : (ii > nx - 1 ? nx - 1 : ii);
      S[b][a] = U[jj * nx + ii];
    }
  }
  const double u = S[2][2];
  double ss = 0.0;
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      S[b][a] -= u;
      ss += S[b][a] * S[b][a];
    }
  const double sigma = sqrt(ss / 24.0);
  double gsrc = st[9];
  for (int q = 0; q < src.ns; ++q) gsrc += time_factor(src, q, t_n) * st[10 + q];
  const double a_ = st[2], b_ = st[3], c_ = st[4], d_ = st[5], ph = st[6];
  const double kappa = a_ + b_ + fabs(c_) + fabs(d_) + fabs(ph);
  f.F0 = a_ * (S[2][3] + S[2][1]) + b_ * (S[3][2] + S[1][2]) - c_ * (S[2][3] - S[2][1]) / 2.0 -
         d_ * (S[3][2] - S[1][2]) / 2.0 + ph * u + gsrc;
  f.s = kappa * sigma + 1e-3 * (fabs(gsrc) + fabs(ph * u));
  f.u = u;
  f.node = j * nx + i;
  const double inv = sigma > 0.0 ? 1.0 / sigma : 0.0;
  int q = 0;
#pragma unroll
  for (int b = 0; b < 5; ++b)
#pragma unroll
    for (int a = 0; a < 5; ++a)
      if (a != 2 || b != 2) f.x[q++] = (float)(S[b][a] * inv);
  const double au = fabs(u) + sigma;
  f.x[24] = (float)(au > 0.0 ? u / au : 0.0);
  const double ik = kappa > 0.0 ? 1.0 / kappa : 0.0;
  f.x[25] = (float)(a_ * ik);
  f.x[26] = (float)(b_ * ik);
  f.x[27] = (float)(c_ * ik);
  f.x[28] = (float)(d_ * ik);
  f.x[29] = (float)(ph * ik);
  const double den = kappa * au;
  const double qq = den > 0.0 ? gsrc / den : 0.0;
  f.x[30] = (float)(qq / (1.0 + fabs(qq)));
  // micro cell Peclet numbers |nu| dxi / (2 alpha), |omega| deta / (2 gamma), squashed
  const double pex = a_ > 0.0 ? fabs(c_) * st[7] / (2.0 * a_) : 0.0;
  const double pee = b_ > 0.0 ? fabs(d_) * st[8] / (2.0 * b_) : 0.0;
  f.x[31] = (float)(pex / (1.0 + pex));
  f.x[32] = (float)(pee / (1.0 + pee));
}

// Inputs of every patch; with U_np1 also the training target of the step U -> U_np1,
// y = (F - F0) / s clipped to [-10, 10] with F = (U_np1 - U) / dt_macro at the node.
__global__ void k_closure_features(Geo g, SrcInfo src, const double* __restrict__ st,
                                   const double* __restrict__ U, double t_n,
                                   float* __restrict__ X, double* __restrict__ F0,
                                   double* __restrict__ sc, const double* __restrict__ Unp1,
                                   double dtm, float* __restrict__ y) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.P) return;
  Feat f;
  closure_features(g, src, st + (long long)p * CL_NST, U, t_n, f);
  for (int q = 0; q < CL_FEAT; ++q) X[(long long)p * CL_FEAT + q] = f.x[q];
  if (F0) F0[p] = f.F0;
  if (sc) sc[p] = f.s;
  if (y) {
    const double F = (Unp1[f.node] - f.u) / dtm;
    double t = f.s > 0.0 ? (F - f.F0) / f.s : 0.0;
    t = t > 10.0 ? 10.0 : (t < -10.0 ? -10.0 : t);
    y[p] = (float)t;
  }
}

// ------------------------------------------------------------------------- training

__device__ __forceinline__ float gelu_f(float x) {
  return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
}
// GELU for inference: erf by the rational-exponential form of Abramowitz and Stegun
// (eq. 7.1.26, |error| <= 1.5e-7 on x >= 0, odd extension), with the hardware reciprocal and
// base-2 exponential: about a third of the instructions of the library erf, and far below
// the bfloat16 rounding the activations get next.
__device__ __forceinline__ float gelu_infer(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, z, 1.0f));
  float p = fmaf(1.061405429f, t, -1.453152027f);
  p = fmaf(p, t, 1.421413741f);
  p = fmaf(p, t, -0.284496736f);
  p = fmaf(p, t, 0.254829592f);
  p *= t;
  const float e = __builtin_amdgcn_exp2f(-z * z * 1.4426950408889634f);
  const float erfz = fmaf(-p, e, 1.0f);  // erf(|x| / sqrt 2)
  return 0.5f * x * (1.0f + copysignf(erfz, x));
}
__device__ __forceinline__ float gelu_grad_f(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) +
         x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// C[M][N] (ldc) = beta C + A B, A = M x K (row-major, or its transpose stored K x M when
// ta), B = K x N (or N x K when tb).  64 x 64 tiles, 256 threads of 4 x 4 outputs.
// Split K: block z sums k in [z kc, (z + 1) kc) into its own slice C + z * cz (the caller
// reduces the slices in a fixed order); one slice (kc >= K, cz = 0) is the plain product.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float* __restrict__ A,
                                              int lda, int ta, const float* __restrict__ B,
                                              int ldb, int tb, float* __restrict__ C, int ldc,
                                              float beta, int kc, long long cz) {
  __shared__ float As[16][65], Bs[16][65];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kb = blockIdx.z * kc, ke = K < kb + kc ? K : kb + kc;
  C += blockIdx.z * cz;
  float acc[4][4] = {};
  for (int k0 = kb; k0 < ke; k0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int kk = e >> 6, mm = e & 63;
      const int gm = m0 + mm, gk = k0 + kk, gn = n0 + mm;
      As[kk][mm] = (gm < M && gk < ke) ? (ta ? A[(long long)gk * lda + gm] : A[(long long)gm * lda + gk]) : 0.f;
      Bs[kk][mm] = (gn < N && gk < ke) ? (tb ? B[(long long)gn * ldb + gk] : B[(long long)gk * ldb + gn]) : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      float a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fmaf(a[r], b[c], acc[r][c]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gm = m0 + ty * 4 + r, gn = n0 + tx * 4 + c;
      if (gm < M && gn < N) {
        float* o = C + (long long)gm * ldc + gn;
        *o = beta != 0.f ? beta * *o + acc[r][c] : acc[r][c];
      }
    }
}

// C[e] = sum over the S slices part[z][e], z ascending (n = M * N outputs, slices of n).
__global__ void k_splitk_reduce(int n, int S, const float* __restrict__ part,
                                float* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  float acc = part[e];
  for (int z = 1; z < S; ++z) acc += part[(long long)z * n + e];
  C[e] = acc;
}

// H += bias (per column), A = GELU(H); n rows of CL_HID.
__global__ void k_bias_gelu(int n, float* __restrict__ H, const float* __restrict__ bias,
                            float* __restrict__ A) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * CL_HID) return;
  const float h = H[e] + bias[e % CL_HID];
  H[e] = h;
  A[e] = gelu_f(h);
}

// Output head: out = A2 w3 + b3, r = out - y, dout = 2 r / n, and per-row products for
// the gradients; dH2 = dout w3 GELU'(H2).  One wave per row (two columns per lane, a
// cross-lane sum), HEAD_ROWS rows per block; the block adds its rows' squared residuals
// to the loss with one atomic.
constexpr int HEAD_ROWS = 4;
__global__ __launch_bounds__(64 * HEAD_ROWS) void k_head(int n, const float* __restrict__ A2,
                                                         const float* __restrict__ H2,
                                                         const float* __restrict__ par,
                                                         const float* __restrict__ y,
                                                         float* __restrict__ out,
                                                         float* __restrict__ dout,
                                                         float* __restrict__ dH2,
                                                         float* __restrict__ loss) {
  __shared__ float lsum[HEAD_ROWS];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x * HEAD_ROWS + w;
  const float* w3 = par + CL_OW3;
  float o = 0.f, sq = 0.f;
  if (r < n) {
    float v = 0.f;
#pragma unroll
    for (int h = 0; h < CL_HID / 64; ++h) {
      const int c = lane + 64 * h;
      v += A2[(long long)r * CL_HID + c] * w3[c];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    o = v + par[CL_OB3];
    if (out && lane == 0) out[r] = o;
    if (y) {
      const float res = o - y[r];
      const float d = 2.0f * res / (float)n;
      if (lane == 0) dout[r] = d;
      sq = res * res / (float)n;
#pragma unroll
      for (int h = 0; h < CL_HID / 64; ++h) {
        const int c = lane + 64 * h;
        dH2[(long long)r * CL_HID + c] = d * w3[c] * gelu_grad_f(H2[(long long)r * CL_HID + c]);
      }
    }
  }
  if (lane == 0) lsum[w] = sq;
  __syncthreads();
  if (y && threadIdx.x == 0) {
    float t = 0.f;
    for (int k = 0; k < HEAD_ROWS; ++k) t += lsum[k];
    atomicAdd(loss, t);
  }
}

// dH1 = dA1 GELU'(H1) in place.
__global__ void k_gelu_back(int n, float* __restrict__ dA, const float* __restrict__ H) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * CL_HID) return;
  dA[e] *= gelu_grad_f(H[e]);
}

// Column sums of n rows (bias gradients) and the output-layer gradients
// dw3 = A2^T dout, db3 = sum dout.  Block c handles column c (c == CL_HID: db3 / b-sums).
__global__ void k_colsums(int n, const float* __restrict__ dH1, const float* __restrict__ dH2,
                          const float* __restrict__ A2, const float* __restrict__ dout,
                          float* __restrict__ grad) {
  __shared__ float r1[256], r2[256], r3[256];
  const int c = blockIdx.x;
  float s1 = 0.f, s2 = 0.f, s3 = 0.f;
  for (int r = threadIdx.x; r < n; r += 256) {
    if (c < CL_HID) {
      s1 += dH1[(long long)r * CL_HID + c];
      s2 += dH2[(long long)r * CL_HID + c];
      s3 += A2[(long long)r * CL_HID + c] * dout[r];
    } else {
      s3 += dout[r];
    }
  }
  r1[threadIdx.x] = s1;
  r2[threadIdx.x] = s2;
  r3[threadIdx.x] = s3;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      r1[threadIdx.x] += r1[threadIdx.x + w];
      r2[threadIdx.x] += r2[threadIdx.x + w];
      r3[threadIdx.x] += r3[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (c < CL_HID) {
      grad[CL_OB1 + c] = r1[0];
      grad[CL_OB2 + c] = r2[0];
      grad[CL_OW3 + c] = r3[0];
    } else {
      grad[CL_OB3] = r3[0];
    }
  }
}

// x[e] = v for e < n (a kernel, not a memset: safe inside captured graphs).
__global__ void k_fill_f32(float* __restrict__ x, long long n, float v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] = v;
}

// Adam on the flat parameter vector (FP32 master weights); step counts from 1.
__global__ void k_adam(float* __restrict__ par, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int step, float lr, float b1, float b2,
                       float eps) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= CL_NPAR) return;
  const float gi = g[e];
  const float mi = b1 * m[e] + (1.f - b1) * gi;
  const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  const float mh = mi / (1.f - powf(b1, (float)step));
  const float vh = vi / (1.f - powf(b2, (float)step));
  par[e] -= lr * mh / (sqrtf(vh) + eps);
}

// Per-feature mean and standard deviation of n rows (two passes in FP64, one block per
// feature); the deviation has a floor of 1e-6.
__global__ void k_colstats(long long n, const float* __restrict__ X, float* __restrict__ mu,
                           float* __restrict__ sd) {
  __shared__ double red[256];
  const int c = blockIdx.x;
  double s = 0.0;
  for (long long r = threadIdx.x; r < n; r += 256) s += X[r * CL_FEAT + c];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (long long r = threadIdx.x; r < n; r += 256) {
    const double d = X[r * CL_FEAT + c] - mean;
    q += d * d;
  }
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mu[c] = (float)mean;
    const double var = red[0] / (double)n;
    sd[c] = (float)sqrt(var > 1e-12 ? var : 1e-12);
  }
}

// Xn = (X - mu) / sd, optionally gathering rows through an affine permutation
// row(r) = (a r + c) mod n_src (a coprime to n_src): a cheap seeded shuffle.
// Targets are standardised with ys = {mean, deviation}.
__global__ void k_standardise(long long n, const float* __restrict__ X, long long n_src,
                              long long a, long long c, const float* __restrict__ mu,
                              const float* __restrict__ sd, float* __restrict__ Xn,
                              const float* __restrict__ y, float* __restrict__ yb,
                              const float* __restrict__ ys) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * CL_FEAT) return;
  const long long r = e / CL_FEAT;
  const int q = (int)(e - r * CL_FEAT);
  const long long src = n_src > 0 ? (a * r + c) % n_src : r;
  Xn[e] = (X[src * CL_FEAT + q] - mu[q]) / sd[q];
  if (yb && q == 0) yb[r] = (y[src] - ys[0]) / ys[1];
}

// Mean and deviation (floor 1e-12) of n targets, one block.
__global__ void k_target_stats(long long n, const float* __restrict__ y, float* __restrict__ ys) {
  __shared__ double red[256];
  double s = 0.0;
  for (long long r = threadIdx.x; r < n; r += 256) s += y[r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double mean = red[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (long long r = threadIdx.x; r < n; r += 256) q += (y[r] - mean) * (y[r] - mean);
  red[threadIdx.x] = q;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double var = red[0] / (double)n;
    ys[0] = (float)mean;
    ys[1] = (float)sqrt(var > 1e-24 ? var : 1e-24);
  }
}

// ------------------------------------------------------------------------- inference

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ unsigned short to_bf16(float x) {
  unsigned int b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);  // nearest, ties to even
  return (unsigned short)(b >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) {
  return __uint_as_float((unsigned int)h << 16);
}

constexpr int K1P = CL_K1P;
// LDS row strides (bfloat16 entries) of the input and hidden tiles, padded by four so that
// the 32 rows one MFMA operand read spans fall on different banks.
constexpr int XS = K1P + 4, HS = CL_HID + 4;

// Packed bfloat16 weights: W1t [CL_HID][K1P] and W2t [CL_HID][CL_HID] (output-major, the
// reduction index contiguous), w3 [CL_HID].
__global__ void k_pack(const float* __restrict__ par, unsigned short* __restrict__ w1t,
                       unsigned short* __restrict__ w2t, unsigned short* __restrict__ w3) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < CL_HID * K1P) {
    const int n = e / K1P, k = e - n * K1P;
    w1t[e] = k < CL_FEAT ? to_bf16(par[CL_OW1 + k * CL_HID + n]) : (unsigned short)0;
  }
  if (e < CL_HID * CL_HID) {
    const int n = e / CL_HID, k = e - n * CL_HID;
    w2t[e] = to_bf16(par[CL_OW2 + k * CL_HID + n]);
  }
  if (e < CL_HID) w3[e] = to_bf16(par[CL_OW3 + e]);
}


// The network on a tile of 64 rows.  xt: LDS [64][XS] bfloat16 inputs (K1P used); ht: LDS
// [64][HS] bfloat16 scratch (CL_HID used); part: LDS [2][64] floats; out: LDS [64] floats (results).  256 threads:
// wave w computes rows 32 (w & 1) .. + 31 and columns 64 (w >> 1) .. + 63 of each layer with
// 32x32x8 MFMA tiles; lane l holds A(row l % 32, k 4 (l / 32) .. + 3), B(k 4 (l / 32) .. + 3,
// col l % 32) and accumulator entry e at row 8 (e / 4) + 4 (l / 32) + e % 4, col l % 32.
__device__ __forceinline__ void mlp_tile(const MlpW& W, const unsigned short* xt,
                                         unsigned short* ht, float* part, float* out) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int mt = w & 1, nh = w >> 1;
  const int li = lane & 31, lk = (lane >> 5) * 4;
  f32x16 acc[2];
  // layer 1
#pragma unroll
  for (int t = 0; t < 2; ++t) acc[t] = f32x16{};
#pragma unroll
  for (int ks = 0; ks < K1P / 8; ++ks) {
    const bf16x4 a = *reinterpret_cast<const bf16x4*>(xt + (32 * mt + li) * XS + 8 * ks + lk);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = 64 * nh + 32 * t + li;
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(W.w1t + n * K1P + 8 * ks + lk);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int col = 64 * nh + 32 * t + li;
    const float bias = W.par[CL_OB1 + col];
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = 32 * mt + 8 * (e / 4) + (lane >> 5) * 4 + (e & 3);
      ht[row * HS + col] = to_bf16(gelu_infer(acc[t][e] + bias));
    }
  }
  __syncthreads();
  // layer 2
#pragma unroll
  for (int t = 0; t < 2; ++t) acc[t] = f32x16{};
#pragma unroll 4
  for (int ks = 0; ks < CL_HID / 8; ++ks) {
    const bf16x4 a = *reinterpret_cast<const bf16x4*>(ht + (32 * mt + li) * HS + 8 * ks + lk);
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int n = 64 * nh + 32 * t + li;
      const bf16x4 b = *reinterpret_cast<const bf16x4*>(W.w2t + n * CL_HID + 8 * ks + lk);
      acc[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc[t], 0, 0, 0);
    }
  }
  // output layer: sum over columns of GELU(h2) w3, per row
  float rs[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) rs[e] = 0.f;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int col = 64 * nh + 32 * t + li;
    const float bias = W.par[CL_OB2 + col], w3 = from_bf16(W.w3[col]);
#pragma unroll
    for (int e = 0; e < 16; ++e) rs[e] += gelu_infer(acc[t][e] + bias) * w3;
  }
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    float v = rs[e];
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    rs[e] = v;
  }
  if (li == 0) {
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const int row = 32 * mt + 8 * (e / 4) + (lane >> 5) * 4 + (e & 3);
      part[nh * 64 + row] = rs[e];
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) out[threadIdx.x] = part[threadIdx.x] + part[64 + threadIdx.x] + W.par[CL_OB3];
  __syncthreads();
}

// Network outputs for standardised rows Xn [n][33] (64 rows per block).
__global__ __launch_bounds__(256) void k_mlp_infer(long long n, const float* __restrict__ Xn,
                                                   MlpW W, float* __restrict__ out) {
  __shared__ __align__(16) unsigned short xt[64 * XS];
  __shared__ __align__(16) unsigned short ht[64 * HS];
  __shared__ float part[128], res[64];
  const long long r0 = (long long)blockIdx.x * 64;
  for (int e = threadIdx.x; e < 64 * K1P; e += 256) {
    const int r = e / K1P, k = e - r * K1P;
    const long long gr = r0 + r;
    xt[r * XS + k] = (k < CL_FEAT && gr < n) ? to_bf16(Xn[gr * CL_FEAT + k]) : (unsigned short)0;
  }
  __syncthreads();
  mlp_tile(W, xt, ht, part, res);
  if (threadIdx.x < 64 && r0 + threadIdx.x < n) out[r0 + threadIdx.x] = res[threadIdx.x];
}

// The closure macro step for groups of 64 patches: features, standardisation, network,
// F_hat = F0 + s y_hat, U_np1 = U + dt_macro F_hat at the patch node (and F_hat stored).
// Single grid: the instance is passed by value and block b takes patches 64 b ..; batch:
// block b takes item b = (instance, first patch) and the instance's tables, with the
// macro step, buffers and Dirichlet values from the shared clock as in the batch kernel.

// Closure macro step: each wave takes one unit of 64 patches (a batch item, or patches
// 64 u .. 64 u + 63 of the single grid), gathers and standardises their inputs, the block
// runs the network on its four 64-row tiles (MFMA), and each wave writes its patches'
// projected values.
__global__ __launch_bounds__(256) void k_closure_step(ClosureArgs Cl) {
  __shared__ __align__(16) unsigned short xt[4 * 64 * XS];
  __shared__ __align__(16) unsigned short ht[64 * HS];
  __shared__ float part[128], res[4 * 64];
  __shared__ double sF0[4 * 64], sS[4 * 64], sU[4 * 64];
  __shared__ int sNode[4 * 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const bool batch = Cl.inst != nullptr;
  const int unit = blockIdx.x * 4 + w;
  const bool valid = unit < Cl.n_items;
  const int inst = batch && valid ? Cl.items[2 * unit] : 0;
  const long long p0 = batch ? (valid ? Cl.items[2 * unit + 1] : 0) : 64LL * unit;
  const BurstArgs& A = batch ? Cl.inst[inst] : Cl.one;
  const double* st = batch ? Cl.st_tab[inst] : Cl.st_one;
  double* fhat = batch ? Cl.fhat_tab[inst] : Cl.fhat_one;
  const double* Uin = A.U;
  double* Uout = A.Unew;
  double t_n = A.t_n;
  if (A.clk != nullptr) {
    const long long n = A.clk->base + Cl.k;
    Uin = (n & 1) ? A.Unew : A.U;
    Uout = (n & 1) ? const_cast<double*>(A.U) : A.Unew;
    t_n = A.t_n + (double)n * A.dt_macro;
    if (valid && p0 == 0 && A.bvals != nullptr) {  // Dirichlet nodes at t_n + dt_macro
      const double* bv = A.bvals + (long long)Cl.k * A.nb;
      for (int q = lane; q < A.nb; q += 64) {
        int i, j;
        boundary_node(A.g, q, i, j);
        Uout[j * A.g.n_xi + i] = bv[q];
      }
    }
  }
  const int r = w * 64 + lane;
  const long long p = p0 + lane;
  const bool mine = valid && p < A.g.P;
  unsigned short* xr = xt + r * XS;
  if (mine) {
    Feat f;
    closure_features(A.g, A.src, st + p * CL_NST, Uin, t_n, f);
#pragma unroll
    for (int q = 0; q < K1P; ++q)
      xr[q] = q < CL_FEAT ? to_bf16((f.x[q] - Cl.mu[q]) / Cl.sd[q]) : (unsigned short)0;
    sF0[r] = f.F0;
    sS[r] = f.s;
    sU[r] = f.u;
    sNode[r] = f.node;
  } else {
    for (int q = 0; q < K1P; ++q) xr[q] = 0;
  }
  __syncthreads();
  for (int tile = 0; tile < 4; ++tile)  // uniform: tiles of units past the end are skipped
    if (blockIdx.x * 4 + tile < Cl.n_items)
      mlp_tile(Cl.W, xt + tile * 64 * XS, ht, part, res + tile * 64);
  if (mine) {
    const double Fh = sF0[r] + sS[r] * ((double)Cl.ys[0] + (double)Cl.ys[1] * (double)res[r]);
    const double un = sU[r] + A.dt_macro * Fh;
    Uout[sNode[r]] = un;
    if (fhat) fhat[p] = Fh;
    if (batch && Cl.sres_tab) Cl.sres_tab[inst][p] = (float)sS[r];
    if (!isfinite(un)) atomicOr(A.flag, 1);
  }
}

}  // namespace

// ----------------------------------------------------------------------------- launchers

hipError_t launch_closure_features(const Geo& g, const SrcInfo& src, const double* st,
                                   const double* U, double t_n, float* X, double* F0,
                                   double* sc, const double* Unp1, double dtm, float* y,
                                   hipStream_t s) {
  hipLaunchKernelGGL(k_closure_features, dim3((g.P + 127) / 128), dim3(128), 0, s, g, src, st,
                     U, t_n, X, F0, sc, Unp1, dtm, y);
  return hipGetLastError();
}

// Workspace of one training step on a batch of nb rows: H1, A1, H2, A2, dH2 (reused as
// dA1 / dH1) [nb][CL_HID], out, dout [nb], grad [CL_NPAR], and CL_SPLITK slices of
// CL_HID x CL_HID partial sums for the weight gradients (whose reduction runs over the nb
// rows: split into up to CL_SPLITK chunks so that they fill the device).
hipError_t launch_mlp_grads(int nb, const float* Xn, const float* y, const float* par,
                            float* H1, float* A1, float* H2, float* A2, float* dH2,
                            float* dH1, float* out, float* dout, float* grad, float* loss,
                            float* part, hipStream_t s) {
  const dim3 blk(256);
  auto gemm = [&](int M, int N, int K, const float* A, int lda, int ta, const float* B, int ldb,
                  int tb, float* C, int ldc) {
    hipLaunchKernelGGL(k_gemm, dim3((N + 63) / 64, (M + 63) / 64, 1), blk, 0, s, M, N, K, A,
                       lda, ta, B, ldb, tb, C, ldc, 0.f, K, 0ll);
  };
  // C (M x N, dense) = A^T B over the nb rows, in S slices of kc rows
  auto gemm_tn_split = [&](int M, int N, const float* A, int lda, const float* B, int ldb,
                           float* C) {
    int S = (nb + 63) / 64;
    if (S > CL_SPLITK) S = CL_SPLITK;
    const int kc = (((nb + S - 1) / S) + 15) / 16 * 16;
    S = (nb + kc - 1) / kc;
    const long long n = (long long)M * N;
    hipLaunchKernelGGL(k_gemm, dim3((N + 63) / 64, (M + 63) / 64, S), blk, 0, s, M, N, nb, A,
                       lda, 1, B, ldb, 0, part, N, 0.f, kc, n);
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)((n + 255) / 256)), blk, 0, s, (int)n, S,
                       part, C);
  };
  const long long nh = (long long)nb * CL_HID;
  const unsigned eb = (unsigned)((nh + 255) / 256);
  gemm(nb, CL_HID, CL_FEAT, Xn, CL_FEAT, 0, par + CL_OW1, CL_HID, 0, H1, CL_HID);
  hipLaunchKernelGGL(k_bias_gelu, dim3(eb), blk, 0, s, nb, H1, par + CL_OB1, A1);
  gemm(nb, CL_HID, CL_HID, A1, CL_HID, 0, par + CL_OW2, CL_HID, 0, H2, CL_HID);
  hipLaunchKernelGGL(k_bias_gelu, dim3(eb), blk, 0, s, nb, H2, par + CL_OB2, A2);
  hipLaunchKernelGGL(k_head, dim3((nb + HEAD_ROWS - 1) / HEAD_ROWS), dim3(64 * HEAD_ROWS), 0, s,
                     nb, A2, H2, par, y, out, dout, dH2, loss);
  if (!y) return hipGetLastError();
  // dW2 = A1^T dH2; dA1 = dH2 W2^T; dH1 = dA1 GELU'(H1); dW1 = Xn^T dH1
  gemm_tn_split(CL_HID, CL_HID, A1, CL_HID, dH2, CL_HID, grad + CL_OW2);
  gemm(nb, CL_HID, CL_HID, dH2, CL_HID, 0, par + CL_OW2, CL_HID, 1, dH1, CL_HID);
  hipLaunchKernelGGL(k_gelu_back, dim3(eb), blk, 0, s, nb, dH1, H1);
  gemm_tn_split(CL_FEAT, CL_HID, Xn, CL_FEAT, dH1, CL_HID, grad + CL_OW1);
  hipLaunchKernelGGL(k_colsums, dim3(CL_HID + 1), blk, 0, s, nb, dH1, dH2, A2, dout, grad);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* x, long long n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, n, v);
  return hipGetLastError();
}

hipError_t launch_adam(float* par, float* m, float* v, const float* g, int step, float lr,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((CL_NPAR + 255) / 256), dim3(256), 0, s, par, m, v, g, step, lr,
                     0.9f, 0.999f, 1e-8f);
  return hipGetLastError();
}

hipError_t launch_colstats(long long n, const float* X, float* mu, float* sd, hipStream_t s) {
  hipLaunchKernelGGL(k_colstats, dim3(CL_FEAT), dim3(256), 0, s, n, X, mu, sd);
  return hipGetLastError();
}

hipError_t launch_standardise(long long n, const float* X, long long n_src, long long a,
                              long long c, const float* mu, const float* sd, float* Xn,
                              const float* y, float* yb, const float* ys, hipStream_t s) {
  const long long e = n * CL_FEAT;
  hipLaunchKernelGGL(k_standardise, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, n, X,
                     n_src, a, c, mu, sd, Xn, y, yb, ys);
  return hipGetLastError();
}

hipError_t launch_target_stats(long long n, const float* y, float* ys, hipStream_t s) {
  hipLaunchKernelGGL(k_target_stats, dim3(1), dim3(256), 0, s, n, y, ys);
  return hipGetLastError();
}

hipError_t launch_pack(const float* par, unsigned short* w1t, unsigned short* w2t,
                       unsigned short* w3, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3((CL_HID * CL_HID + 255) / 256), dim3(256), 0, s, par, w1t,
                     w2t, w3);
  return hipGetLastError();
}

hipError_t launch_mlp_infer(long long n, const float* Xn, const unsigned short* w1t,
                            const unsigned short* w2t, const unsigned short* w3, const float* par,
                            float* out, hipStream_t s) {
  MlpW W{w1t, w2t, w3, par};
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((n + 63) / 64)), dim3(256), 0, s, n, Xn, W,
                     out);
  return hipGetLastError();
}

hipError_t launch_closure_step(const ClosureArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_closure_step, dim3((a.n_items + 3) / 4), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace pdk
