// Learned warm start: a small convolutional encoder-decoder mapping the
// forcings and frequency encodings of a problem to an initial guess for the N_f
// filtered fields.  Not part of the paper's method; the initial guess only
// changes where GMRES starts (a zero start is the fallback).
//
// Compute: every 3x3 convolution (forward, backward w.r.t. input and weights)
// is an implicit GEMM on the matrix cores: im2col into bfloat16, then one
// BF16 MFMA GEMM kernel (v_mfma_f32_16x16x32_bf16, float32 accumulation),
// col2im for the input gradient.  Activations, gradients and master weights
// are float32 in NHWC layout [B][H][W][C]; the K index of a convolution is
// k = (ky*3 + kx)*Cin + ci so each im2col row reads contiguous channels.
// Network (matches the float64 reference):
//   a1 = relu(conv(x))            C0 -> 32          (H, W)
//   a2 = relu(conv_s2(a1))        32 -> 64          (H/2)
//   a3 = relu(conv_s2(a2))        64 -> 64          (H/4)
//   a4 = relu(conv(up2(a3))) + a2 64 -> 64          (H/2)
//   a5 = relu(conv(up2(a4))) + a1 64 -> 32          (H)
//   y  = conv(a5)                 32 -> N_f         (H)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/mfwh.h"

namespace mfwh {
namespace cnn {

typedef short bf16raw;
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16raw f2bf(float f) {
  // round to nearest even
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16raw)(u >> 16);
}

// ---------------------------------------------------------------------------
// C (float32, [M][N] row-major, split-K partial z) = A (bf16) * B (bf16)
//   A: [M][K] row-major (ATRANS = 0) or stored as [K][M] (ATRANS = 1)
//   B: [K][N] row-major
// Block 256 threads = 4 waves, block tile 64 x 64, each wave 32 x 32 as
// 2 x 2 tiles of gfx950's v_mfma_f32_16x16x32_bf16; K advances by 32.
// Staging: every thread moves one 16-byte group of 8 bf16 per operand per K
// step (global dwordx4 loads when the group is in range and 16-byte
// aligned, element loads otherwise).  In LDS both operands are stored
// k-contiguous (As[m][k], Bt[n][k]) so that each lane reads its 8 MFMA
// operand values as one 16-byte LDS load; rows are padded by 8 bf16 so the
// 16 rows a wave reads start in different banks.  The lanes of an MFMA
// operand hold rows (A) / columns (B) lane % 16 and the k-group lane / 16;
// A and B use the same k-group assignment, so any k order the instruction
// pairs them in gives the same sum.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x8 __attribute__((ext_vector_type(8)));

template <int ATRANS>
__global__ void __launch_bounds__(256) k_gemm_bf16(const bf16raw* __restrict__ A,
                                                   const bf16raw* __restrict__ B,
                                                   float* __restrict__ C, int M, int N, int K,
                                                   int lda, int ldb, int ldc, int kchunk,
                                                   long long zstride) {
  constexpr int KT = 32, PAD = 8;
  __shared__ __align__(16) bf16raw As[64][KT + PAD];
  __shared__ __align__(16) bf16raw Bt[64][KT + PAD];
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int m0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int wm = (wave & 1) * 32, wn = (wave >> 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += KT) {
    s16x8 va, vb;
    if (!ATRANS) {
      // A [M][K]: thread -> row r, k group g (8 consecutive k)
      const int r = tid >> 2, g = (tid & 3) * 8;
      const int gm = m0 + r, gk = k0 + g;
      const bf16raw* src = A + (long long)gm * lda + gk;
      if (gm < M && gk + 8 <= kend && (((uintptr_t)src) & 15) == 0) {
        va = *(const s16x8*)src;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) va[j] = (gm < M && gk + j < kend) ? src[j] : (bf16raw)0;
      }
      *(s16x8*)&As[r][g] = va;
    } else {
      // A stored [K][M]: thread -> k row kk, m group g (8 consecutive m)
      const int kk = tid >> 3, g = (tid & 7) * 8;
      const int gk = k0 + kk, gm = m0 + g;
      const bf16raw* src = A + (long long)gk * lda + gm;
      if (gk < kend && gm + 8 <= M && (((uintptr_t)src) & 15) == 0) {
        va = *(const s16x8*)src;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) va[j] = (gk < kend && gm + j < M) ? src[j] : (bf16raw)0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) As[g + j][kk] = va[j];
    }
    {
      // B [K][N]: thread -> k row kk, n group g
      const int kk = tid >> 3, g = (tid & 7) * 8;
      const int gk = k0 + kk, gn = n0 + g;
      const bf16raw* src = B + (long long)gk * ldb + gn;
      if (gk < kend && gn + 8 <= N && (((uintptr_t)src) & 15) == 0) {
        vb = *(const s16x8*)src;
      } else {
#pragma unroll
        for (int j = 0; j < 8; ++j) vb[j] = (gk < kend && gn + j < N) ? src[j] : (bf16raw)0;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) Bt[g + j][kk] = vb[j];
    }
    __syncthreads();
    const int li = lane & 15, lk = (lane >> 4) * 8;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const s16x8 ar = *(const s16x8*)&As[wm + a * 16 + li][lk];
      const bf16x8 av = __builtin_bit_cast(bf16x8, ar);
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const s16x8 br = *(const s16x8*)&Bt[wn + b * 16 + li][lk];
        const bf16x8 bv = __builtin_bit_cast(bf16x8, br);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // C layout of one 16x16 tile: lane holds column (lane % 16), rows 4*(lane/16) + i
  float* Cz = C + blockIdx.z * zstride;
  const int col = lane & 15, rb = (lane >> 4) * 4;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int gm = m0 + wm + a * 16 + rb + i, gn = n0 + wn + b * 16 + col;
        if (gm < M && gn < N) Cz[(long long)gm * ldc + gn] = acc[a][b][i];
      }
}

__global__ void __launch_bounds__(256) k_splitk_reduce(const float* __restrict__ P, int nz,
                                                       long long n, float* __restrict__ C) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    float s = 0.f;
    for (int z = 0; z < nz; ++z) s += P[z * n + i];
    C[i] = s;
  }
}

// ---------------------------------------------------------------------------
// im2col: col[p][k] (bf16, row length ldk >= 9*Cin, zero padded) for a 3x3
// convolution with padding 1 and stride s over input x (NHWC float32,
// Hi x Wi x Cin).  up = 1 reads x through nearest up-sampling to (Hu, Wu)
// (x is then (Hu+1)/2 x (Wu+1)/2).  Output positions: Ho x Wo.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_im2col(const float* __restrict__ x, int B, int Hi,
                                                int Wi, int Cin, int stride, int up, int Hu,
                                                int Wu, int Ho, int Wo, int ldk,
                                                bf16raw* __restrict__ col) {
  const long long total = (long long)B * Ho * Wo * ldk;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const int k = (int)(t % ldk);
    const long long p = t / ldk;
    float v = 0.f;
    if (k < 9 * Cin) {
      const int ci = k % Cin, tap = k / Cin, ky = tap / 3, kx = tap % 3;
      const int xo = (int)(p % Wo);
      const int yo = (int)((p / Wo) % Ho);
      const int b = (int)(p / ((long long)Wo * Ho));
      const int iy = stride * yo + ky - 1, ix = stride * xo + kx - 1;
      const int Hs = up ? Hu : Hi, Ws = up ? Wu : Wi;
      if (iy >= 0 && iy < Hs && ix >= 0 && ix < Ws) {
        const int sy = up ? iy / 2 : iy, sx = up ? ix / 2 : ix;
        v = x[(((long long)b * Hi + sy) * Wi + sx) * Cin + ci];
      }
    }
    col[t] = f2bf(v);
  }
}

// col2im (gather): dx[b][iy][ix][ci] = sum over taps of dcol[p(y,x)][k] with
// stride*y + ky - 1 = iy, stride*x + kx - 1 = ix.  dx is Hs x Ws (the
// up-sampled size when the layer reads an up-sampled input).
__global__ void __launch_bounds__(256) k_col2im(const float* __restrict__ dcol, int B, int Hs,
                                                int Ws, int Cin, int stride, int Ho, int Wo,
                                                int ldk, float* __restrict__ dx) {
  const long long total = (long long)B * Hs * Ws * Cin;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const int ci = (int)(t % Cin);
    const int ix = (int)((t / Cin) % Ws);
    const int iy = (int)((t / ((long long)Cin * Ws)) % Hs);
    const int b = (int)(t / ((long long)Cin * Ws * Hs));
    float s = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
      const int ny = iy + 1 - ky;
      if (ny < 0 || ny % stride) continue;
      const int yo = ny / stride;
      if (yo >= Ho) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int nx = ix + 1 - kx;
        if (nx < 0 || nx % stride) continue;
        const int xo = nx / stride;
        if (xo >= Wo) continue;
        const long long p = ((long long)b * Ho + yo) * Wo + xo;
        s += dcol[p * ldk + (ky * 3 + kx) * Cin + ci];
      }
    }
    dx[t] = s;
  }
}

// dA (half resolution, Ha x Wa) = sum of the 2x2 block of dU (Hu x Wu)
__global__ void __launch_bounds__(256) k_up2_bwd(const float* __restrict__ du, int B, int Hu,
                                                 int Wu, int C, int Ha, int Wa,
                                                 float* __restrict__ da) {
  const long long total = (long long)B * Ha * Wa * C;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const int c = (int)(t % C);
    const int x = (int)((t / C) % Wa);
    const int y = (int)((t / ((long long)C * Wa)) % Ha);
    const int b = (int)(t / ((long long)C * Wa * Ha));
    float s = 0.f;
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const int uy = 2 * y + dy, ux = 2 * x + dx;
        if (uy < Hu && ux < Wu) s += du[(((long long)b * Hu + uy) * Wu + ux) * C + c];
      }
    da[t] = s;
  }
}

// z = gemm + bias; a = relu(z) (+ skip); act = 0: a = z (no relu)
__global__ void __launch_bounds__(256) k_bias_act(const float* __restrict__ g,
                                                  const float* __restrict__ bias, long long P,
                                                  int C, int act, const float* __restrict__ skip,
                                                  float* __restrict__ z, float* __restrict__ a) {
  const long long n = P * C;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
       t += (long long)gridDim.x * 256) {
    const float v = g[t] + bias[t % C];
    if (z) z[t] = v;
    float r = act ? fmaxf(v, 0.f) : v;
    if (skip) r += skip[t];
    a[t] = r;
  }
}

// dz = da * (z > 0), also a bf16 copy padded to ldz columns
__global__ void __launch_bounds__(256) k_relu_bwd(const float* __restrict__ da,
                                                  const float* __restrict__ z, long long P, int C,
                                                  int relu, float* __restrict__ dz,
                                                  bf16raw* __restrict__ dzb, int ldz) {
  const long long n = P * ldz;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
       t += (long long)gridDim.x * 256) {
    const int c = (int)(t % ldz);
    const long long p = t / ldz;
    float v = 0.f;
    if (c < C) {
      const long long s = p * C + c;
      v = relu ? (z[s] > 0.f ? da[s] : 0.f) : da[s];
      dz[s] = v;
    }
    dzb[t] = f2bf(v);
  }
}

__global__ void __launch_bounds__(256) k_add(float* __restrict__ y, const float* __restrict__ x,
                                             long long n) {
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < n;
       t += (long long)gridDim.x * 256)
    y[t] += x[t];
}

// db[c] = sum_p dz[p][c]   (one block per channel, deterministic)
__global__ void __launch_bounds__(256) k_bias_grad(const float* __restrict__ dz, long long P,
                                                   int C, float* __restrict__ db) {
  __shared__ float sh[256];
  const int c = blockIdx.x;
  float s = 0.f;
  for (long long p = threadIdx.x; p < P; p += 256) s += dz[p * C + c];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) db[c] = sh[0];
}

// loss partials and dy = 2 (y - t) / n
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ y,
                                             const float* __restrict__ t, long long n,
                                             float* __restrict__ dy, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    const float d = y[i] - t[i];
    dy[i] = 2.f * d / (float)n;
    s += (double)d * d;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// t[b][:] /= rms(t[b][:]) for every sample b (one block per sample)
__global__ void __launch_bounds__(256) k_normalize(float* __restrict__ t, long long per) {
  __shared__ double sh[256];
  float* tb = t + (long long)blockIdx.x * per;
  double s = 0.0;
  for (long long i = threadIdx.x; i < per; i += 256) s += (double)tb[i] * tb[i];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double rms = sqrt(sh[0] / (double)per);
  const float inv = rms > 0 ? (float)(1.0 / rms) : 0.f;
  for (long long i = threadIdx.x; i < per; i += 256) tb[i] *= inv;
}

// weight (cout, cin, 3, 3) float32 -> Wt[k][co] (ldn columns) and
// WtT[co][k] (ldk columns) in bf16, k = (ky*3+kx)*cin + ci, zero padded
__global__ void __launch_bounds__(256) k_pack_w(const float* __restrict__ W, int cout, int cin,
                                                int kp, int np, bf16raw* __restrict__ Wt,
                                                bf16raw* __restrict__ WtT) {
  const int total = kp * np;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < total; t += gridDim.x * 256) {
    const int k = t / np, co = t % np;
    float v = 0.f;
    if (k < 9 * cin && co < cout) {
      const int ci = k % cin, tap = k / cin;
      v = W[(co * cin + ci) * 9 + tap];
    }
    const bf16raw b = f2bf(v);
    Wt[t] = b;
    WtT[(long long)co * kp + k] = b;
  }
}

// dWt[k][co] (ld np) -> dW (cout, cin, 3, 3)
__global__ void __launch_bounds__(256) k_unpack_dw(const float* __restrict__ dWt, int cout,
                                                   int cin, int np, float* __restrict__ dW) {
  const int total = cout * cin * 9;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < total; t += gridDim.x * 256) {
    const int tap = t % 9, ci = (t / 9) % cin, co = t / (9 * cin);
    dW[t] = dWt[(tap * cin + ci) * np + co];
  }
}

__global__ void __launch_bounds__(256) k_adam(float* __restrict__ p, const float* __restrict__ g,
                                              float* __restrict__ m, float* __restrict__ v,
                                              long long n, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (long long)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// max |f_m| over the grid for every (b, m): one block each
__global__ void __launch_bounds__(256) k_maxabs(const double* __restrict__ f, long long npix,
                                                double* __restrict__ out) {
  __shared__ double sh[256];
  const double* fb = f + (long long)blockIdx.x * npix;
  double s = 0.0;
  for (long long i = threadIdx.x; i < npix; i += 256) s = fmax(s, fabs(fb[i]));
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = sh[0];
}

// features NHWC [B][H][W][6 nf]: f_m / max|f_m|, sin/cos(omega_m x),
// sin/cos(omega_m y), omega_m / 50
__global__ void __launch_bounds__(256) k_features(const double* __restrict__ f,
                                                  const double* __restrict__ fmax,
                                                  const double* __restrict__ omega, int B, int nf,
                                                  int H, int W, double ly, double lx,
                                                  float* __restrict__ feat) {
  const int C = 6 * nf;
  const long long total = (long long)B * H * W * C;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const int c = (int)(t % C);
    const int x = (int)((t / C) % W);
    const int y = (int)((t / ((long long)C * W)) % H);
    const int b = (int)(t / ((long long)C * W * H));
    const int grp = c / nf, m = c % nf;
    const double om = omega[b * nf + m];
    const double X = lx * x / (W - 1), Y = ly * y / (H - 1);
    double v;
    switch (grp) {
      case 0: {
        const double s = fmax[b * nf + m];
        const double fv = f[(((long long)b * nf + m) * H + y) * W + x];
        v = s > 0 ? fv / s : fv;
        break;
      }
      case 1: v = sin(om * X); break;
      case 2: v = cos(om * X); break;
      case 3: v = sin(om * Y); break;
      case 4: v = cos(om * Y); break;
      default: v = om / 50.0; break;
    }
    feat[t] = (float)v;
  }
}

// dir = 0: v[b][m][y][x] (float64, zero boundary) = out[b][y][x][m] * max|f| / omega^2
// dir = 1: out[b][y][x][m] (float32) = v * omega^2 / max|f|   (training targets)
__global__ void __launch_bounds__(256) k_scale(int dir, float* __restrict__ out,
                                               double* __restrict__ v,
                                               const double* __restrict__ fmax,
                                               const double* __restrict__ omega, int B, int nf,
                                               int H, int W) {
  const long long total = (long long)B * nf * H * W;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total;
       t += (long long)gridDim.x * 256) {
    const int x = (int)(t % W);
    const int y = (int)((t / W) % H);
    const int m = (int)((t / ((long long)W * H)) % nf);
    const int b = (int)(t / ((long long)W * H * nf));
    const double om = omega[b * nf + m];
    const double s = fmax[b * nf + m] / (om * om);
    const long long o = (((long long)b * H + y) * W + x) * nf + m;
    if (dir == 0) {
      const bool bnd = x == 0 || y == 0 || x == W - 1 || y == H - 1;
      v[t] = bnd ? 0.0 : (double)out[o] * s;
    } else {
      out[o] = s > 0 ? (float)(v[t] / s) : 0.f;
    }
  }
}

}  // namespace cnn
}  // namespace mfwh

// =============================================================================
// host orchestration
// =============================================================================
namespace mfwh {
namespace cnn {
namespace {

thread_local std::string g_cnn_err;
int cfail(int code, const std::string& m) {
  g_cnn_err = m;
  return code;
}
#define CHIP(...)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (__VA_ARGS__);                                                      \
    if (e_ != hipSuccess)                                                               \
      return cfail(MFWH_EHIP, std::string(#__VA_ARGS__) + ": " + hipGetErrorString(e_)); \
  } while (0)
#define CCHK(...)          \
  do {                     \
    int r_ = (__VA_ARGS__); \
    if (r_ < 0) return r_; \
  } while (0)

constexpr int kC1 = 32, kC2 = 64, kLayers = 6;

struct Layer {
  int cin, cout, stride, up;      // up: reads up2(input)
  int Hi, Wi;                     // stored input size
  int Hs, Ws;                     // size the 3x3 window sees (up-sampled size when up)
  int Ho, Wo;
  int K;                          // 9 * cin
  long long P;                    // batch * Ho * Wo
  size_t woff, boff;              // offsets in the flat parameter vector
};

struct Net {
  int B, nf, H, W, c0;
  int H2, W2, H3, W3;
  Layer L[kLayers];
  size_t nparam;
};

Net make_net(int B, int nf, int H, int W) {
  Net n;
  n.B = B; n.nf = nf; n.H = H; n.W = W; n.c0 = 6 * nf;
  n.H2 = (H - 1) / 2 + 1; n.W2 = (W - 1) / 2 + 1;
  n.H3 = (n.H2 - 1) / 2 + 1; n.W3 = (n.W2 - 1) / 2 + 1;
  auto mk = [&](int cin, int cout, int stride, int up, int Hi, int Wi, int Hs, int Ws, int Ho,
                int Wo) {
    Layer l;
    l.cin = cin; l.cout = cout; l.stride = stride; l.up = up;
    l.Hi = Hi; l.Wi = Wi; l.Hs = Hs; l.Ws = Ws; l.Ho = Ho; l.Wo = Wo;
    l.K = 9 * cin;
    l.P = (long long)B * Ho * Wo;
    l.woff = l.boff = 0;
    return l;
  };
  n.L[0] = mk(n.c0, kC1, 1, 0, H, W, H, W, H, W);
  n.L[1] = mk(kC1, kC2, 2, 0, H, W, H, W, n.H2, n.W2);
  n.L[2] = mk(kC2, kC2, 2, 0, n.H2, n.W2, n.H2, n.W2, n.H3, n.W3);
  n.L[3] = mk(kC2, kC2, 1, 1, n.H3, n.W3, n.H2, n.W2, n.H2, n.W2);
  n.L[4] = mk(kC2, kC1, 1, 1, n.H2, n.W2, H, W, H, W);
  n.L[5] = mk(kC1, nf, 1, 0, H, W, H, W, H, W);
  size_t o = 0;
  for (auto& l : n.L) {
    l.woff = o;
    o += (size_t)l.cout * l.cin * 9;
    l.boff = o;
    o += l.cout;
  }
  n.nparam = o;
  return n;
}

struct Buf {
  float *z[kLayers], *a[kLayers];      // a[5] = y
  bf16raw *col, *wt[kLayers], *wtT[kLayers];
  float *C, *dcol, *part, *dWt, *s1, *s2, *gU, *gD, *dz, *dy;
  bf16raw* dzb;
  double *mse, *fmax;
  size_t bytes;
};

constexpr int kSplit = 64;
constexpr int kMsePart = 1024;

Buf carve_buf(const Net& n, char* base) {
  Buf b;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  long long maxPK = 0, maxPC = 0, maxKC = 0;
  for (int i = 0; i < kLayers; ++i) {
    const Layer& l = n.L[i];
    b.z[i] = (float*)take((size_t)l.P * l.cout * 4);
    b.a[i] = (float*)take((size_t)l.P * l.cout * 4);
    b.wt[i] = (bf16raw*)take((size_t)l.K * l.cout * 2);
    b.wtT[i] = (bf16raw*)take((size_t)l.K * l.cout * 2);
    maxPK = std::max(maxPK, l.P * l.K);
    maxPC = std::max(maxPC, l.P * (long long)l.cout);
    maxKC = std::max(maxKC, (long long)l.K * l.cout);
  }
  const long long P1 = n.L[0].P, P2 = n.L[1].P;
  b.col = (bf16raw*)take((size_t)maxPK * 2);
  b.dcol = (float*)take((size_t)maxPK * 4);
  b.C = (float*)take((size_t)maxPC * 4);
  b.part = (float*)take((size_t)kSplit * maxKC * 4);
  b.dWt = (float*)take((size_t)maxKC * 4);
  b.s1 = (float*)take((size_t)P1 * kC1 * 4);
  b.s2 = (float*)take((size_t)P2 * kC2 * 4);
  b.gU = (float*)take((size_t)P1 * kC2 * 4);
  b.gD = (float*)take((size_t)P1 * kC2 * 4);
  b.dz = (float*)take((size_t)P1 * kC2 * 4);
  b.dy = (float*)take((size_t)P1 * n.nf * 4);
  b.dzb = (bf16raw*)take((size_t)P1 * kC2 * 2);
  b.mse = (double*)take(kMsePart * 8);
  b.fmax = (double*)take((size_t)n.B * n.nf * 8);
  b.bytes = (off + 255) / 256 * 256;
  return b;
}

inline unsigned grid_for(long long n) {
  return (unsigned)std::max<long long>(1, std::min<long long>((n + 255) / 256, 16384));
}

// C[M][N] = A * B (A row-major [M][K] or, with atrans, stored [K][M])
int gemm(bool atrans, const bf16raw* A, const bf16raw* B, float* C, long long M, int N,
         long long K, int lda, int ldb, int ldc, float* part, hipStream_t s) {
  int nz = 1;
  long long kc = (K + 31) / 32 * 32;
  if (atrans && K > 8192) {                  // long reductions: deterministic split-K
    nz = (int)std::min<long long>(kSplit, (K + 4095) / 4096);
    kc = ((K + nz - 1) / nz + 31) / 32 * 32;
    nz = (int)((K + kc - 1) / kc);
  }
  dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64), (unsigned)nz);
  float* out = nz > 1 ? part : C;
  const long long zs = M * (long long)N;
  if (nz > 1 && ldc != N) return cfail(MFWH_EINVAL, "split-K output must be dense");
  if (atrans)
    k_gemm_bf16<1><<<grid, 256, 0, s>>>(A, B, out, (int)M, N, (int)K, lda, ldb, ldc, (int)kc, zs);
  else
    k_gemm_bf16<0><<<grid, 256, 0, s>>>(A, B, out, (int)M, N, (int)K, lda, ldb, ldc, (int)kc, zs);
  CHIP(hipGetLastError());
  if (nz > 1) {
    k_splitk_reduce<<<grid_for(zs), 256, 0, s>>>(part, nz, zs, C);
    CHIP(hipGetLastError());
  }
  return MFWH_OK;
}

int im2col(const Net& n, const Layer& l, const float* x, bf16raw* col, hipStream_t s) {
  const long long tot = l.P * l.K;
  k_im2col<<<grid_for(tot), 256, 0, s>>>(x, n.B, l.Hi, l.Wi, l.cin, l.stride, l.up, l.Hs, l.Ws,
                                          l.Ho, l.Wo, l.K, col);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int check_dims(int B, int nf, int H, int W) {
  if (B < 1 || nf < 1 || nf > MFWH_MAX_NF || H < 4 || W < 4 || (long long)B * H * W > (1LL << 26))
    return cfail(MFWH_EINVAL, "bad network dimensions");
  return MFWH_OK;
}

int forward(const Net& n, const Buf& b, const float* params, const float* feat, hipStream_t s) {
  for (int i = 0; i < kLayers; ++i) {
    const Layer& l = n.L[i];
    const int tot = l.K * l.cout;
    k_pack_w<<<grid_for(tot), 256, 0, s>>>(params + l.woff, l.cout, l.cin, l.K, l.cout, b.wt[i],
                                           b.wtT[i]);
    CHIP(hipGetLastError());
  }
  const float* in[kLayers] = {feat, b.a[0], b.a[1], b.a[2], b.a[3], b.a[4]};
  const float* skip[kLayers] = {nullptr, nullptr, nullptr, b.a[1], b.a[0], nullptr};
  for (int i = 0; i < kLayers; ++i) {
    const Layer& l = n.L[i];
    CCHK(im2col(n, l, in[i], b.col, s));
    CCHK(gemm(false, b.col, b.wt[i], b.C, l.P, l.cout, l.K, l.K, l.cout, l.cout, b.part, s));
    const int act = i < kLayers - 1;
    k_bias_act<<<grid_for(l.P * l.cout), 256, 0, s>>>(b.C, params + l.boff, l.P, l.cout, act,
                                                      skip[i], b.z[i], b.a[i]);
    CHIP(hipGetLastError());
  }
  return MFWH_OK;
}

// weight and bias gradient of layer i given dz (float32 [P][cout]) and its
// bf16 copy; input activation `x`
int layer_wgrad(const Net& n, const Buf& b, int i, const float* x, float* grad, hipStream_t s) {
  const Layer& l = n.L[i];
  CCHK(im2col(n, l, x, b.col, s));
  CCHK(gemm(true, b.col, b.dzb, b.dWt, l.K, l.cout, l.P, l.K, l.cout, l.cout, b.part, s));
  k_unpack_dw<<<grid_for((long long)l.cout * l.cin * 9), 256, 0, s>>>(b.dWt, l.cout, l.cin, l.cout,
                                                                      grad + l.woff);
  CHIP(hipGetLastError());
  k_bias_grad<<<l.cout, 256, 0, s>>>(b.dz, l.P, l.cout, grad + l.boff);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

// input gradient of layer i: dcol = dz * W^T, col2im onto the window grid
int layer_dgrad(const Net& n, const Buf& b, int i, float* dx, hipStream_t s) {
  const Layer& l = n.L[i];
  CCHK(gemm(false, b.dzb, b.wtT[i], b.dcol, l.P, l.K, l.cout, l.cout, l.K, l.K, b.part, s));
  const long long tot = (long long)n.B * l.Hs * l.Ws * l.cin;
  k_col2im<<<grid_for(tot), 256, 0, s>>>(b.dcol, n.B, l.Hs, l.Ws, l.cin, l.stride, l.Ho, l.Wo,
                                         l.K, dx);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int relu_bwd(const Buf& b, const float* da, const float* z, long long P, int C, int relu,
             hipStream_t s) {
  k_relu_bwd<<<grid_for(P * C), 256, 0, s>>>(da, z, P, C, relu, b.dz, b.dzb, C);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

}  // namespace
}  // namespace cnn
}  // namespace mfwh

using namespace mfwh::cnn;

namespace mfwh {
namespace cnn {
namespace {
// One layer as its own net (layer 0) with the buffers the layer helpers use.
struct ConvOne {
  Net n;
  Buf b{};
  size_t bytes = 0;
};

int conv_one(int B, int Hi, int Wi, int cin, int cout, int stride, int up, int Hs, int Ws,
             char* base, ConvOne* c) {
  if (B < 1 || Hi < 1 || Wi < 1 || cin < 1 || cout < 1 || cin > 256 || cout > 256 ||
      (stride != 1 && stride != 2) || (up != 0 && up != 1))
    return cfail(MFWH_EINVAL, "bad convolution dimensions");
  if (!up && (Hs != Hi || Ws != Wi)) return cfail(MFWH_EINVAL, "Hs, Ws must equal Hi, Wi");
  if (up && (Hs < 1 || Ws < 1 || Hs > 2 * Hi || Ws > 2 * Wi))
    return cfail(MFWH_EINVAL, "up-sampled window must fit 2 Hi x 2 Wi");
  if ((long long)B * Hs * Ws > (1LL << 26)) return cfail(MFWH_EINVAL, "layer too large");
  Net& n = c->n;
  n = Net{};
  n.B = B;
  Layer& l = n.L[0];
  l.cin = cin; l.cout = cout; l.stride = stride; l.up = up;
  l.Hi = Hi; l.Wi = Wi; l.Hs = Hs; l.Ws = Ws;
  l.Ho = (Hs - 1) / stride + 1; l.Wo = (Ws - 1) / stride + 1;
  l.K = 9 * cin;
  l.P = (long long)B * l.Ho * l.Wo;
  l.woff = 0;
  l.boff = (size_t)cout * cin * 9;
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    off = (off + 255) / 256 * 256;
    char* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  };
  Buf& b = c->b;
  b.wt[0] = (bf16raw*)take((size_t)l.K * cout * 2);
  b.wtT[0] = (bf16raw*)take((size_t)l.K * cout * 2);
  b.col = (bf16raw*)take((size_t)l.P * l.K * 2);
  b.dcol = (float*)take((size_t)l.P * l.K * 4);
  b.C = (float*)take((size_t)l.P * cout * 4);
  b.part = (float*)take((size_t)kSplit * l.K * cout * 4);
  b.dWt = (float*)take((size_t)l.K * cout * 4);
  b.dz = (float*)take((size_t)l.P * cout * 4);
  b.dzb = (bf16raw*)take((size_t)l.P * cout * 2);
  b.gU = (float*)take((size_t)B * Hs * Ws * cin * 4);
  c->bytes = (off + 255) / 256 * 256;
  return MFWH_OK;
}
}  // namespace
}  // namespace cnn
}  // namespace mfwh

extern "C" {

const char* mfwh_cnn_last_error(void) { return g_cnn_err.c_str(); }

size_t mfwh_cnn_conv3x3_workspace_bytes(int batch, int Hi, int Wi, int cin, int cout, int stride,
                                        int up, int Hs, int Ws) {
  ConvOne c;
  if (conv_one(batch, Hi, Wi, cin, cout, stride, up, Hs, Ws, nullptr, &c) != MFWH_OK) return 0;
  return c.bytes;
}

int mfwh_cnn_conv3x3(int batch, int Hi, int Wi, int cin, int cout, int stride, int up, int Hs,
                     int Ws, const float* x, const float* wb, float* z, const float* dz,
                     float* dx, float* dwb, void* ws, size_t ws_bytes, void* stream) {
  ConvOne c;
  CCHK(conv_one(batch, Hi, Wi, cin, cout, stride, up, Hs, Ws, nullptr, &c));
  if (!ws || ((uintptr_t)ws) % 256) return cfail(MFWH_EWORKSPACE, "workspace null or misaligned");
  if (c.bytes > ws_bytes) return cfail(MFWH_EWORKSPACE, "workspace too small");
  CCHK(conv_one(batch, Hi, Wi, cin, cout, stride, up, Hs, Ws, (char*)ws, &c));
  if (!x || !wb) return cfail(MFWH_EINVAL, "null array");
  if (dz ? (!dx || !dwb) : !z) return cfail(MFWH_EINVAL, "null output array");
  const Net& n = c.n;
  const Buf& b = c.b;
  const Layer& l = n.L[0];
  hipStream_t s = (hipStream_t)stream;
  k_pack_w<<<grid_for((long long)l.K * l.cout), 256, 0, s>>>(wb, l.cout, l.cin, l.K, l.cout,
                                                             b.wt[0], b.wtT[0]);
  CHIP(hipGetLastError());
  if (!dz) {
    CCHK(im2col(n, l, x, b.col, s));
    CCHK(gemm(false, b.col, b.wt[0], b.C, l.P, l.cout, l.K, l.K, l.cout, l.cout, b.part, s));
    k_bias_act<<<grid_for(l.P * l.cout), 256, 0, s>>>(b.C, wb + l.boff, l.P, l.cout, 0, nullptr,
                                                      nullptr, z);
    CHIP(hipGetLastError());
    return MFWH_OK;
  }
  CCHK(relu_bwd(b, dz, nullptr, l.P, l.cout, 0, s));          // dz -> float32 and bf16 copies
  CCHK(layer_wgrad(n, b, 0, x, dwb, s));
  if (!up) {
    CCHK(layer_dgrad(n, b, 0, dx, s));
  } else {
    CCHK(layer_dgrad(n, b, 0, b.gU, s));                        // d up2(x) on the window grid
    k_up2_bwd<<<grid_for((long long)batch * Hi * Wi * cin), 256, 0, s>>>(b.gU, batch, Hs, Ws,
                                                                          cin, Hi, Wi, dx);
    CHIP(hipGetLastError());
  }
  return MFWH_OK;
}

size_t mfwh_cnn_param_count(int nf) {
  if (nf < 1 || nf > MFWH_MAX_NF) return 0;
  return make_net(1, nf, 8, 8).nparam;
}

size_t mfwh_cnn_workspace_bytes(int batch, int nf, int H, int W) {
  if (check_dims(batch, nf, H, W) != MFWH_OK) return 0;
  return carve_buf(make_net(batch, nf, H, W), nullptr).bytes;
}

static int ws_check(const Net& n, void* ws, size_t ws_bytes, Buf* b) {
  if (!ws || ((uintptr_t)ws) % 256) return cfail(MFWH_EWORKSPACE, "workspace null or misaligned");
  *b = carve_buf(n, (char*)ws);
  if (b->bytes > ws_bytes) return cfail(MFWH_EWORKSPACE, "workspace too small");
  return MFWH_OK;
}

int mfwh_cnn_features(int batch, int nf, int H, int W, const double* f, const double* omega,
                      double ly, double lx, float* feat, void* ws, size_t ws_bytes,
                      void* stream) {
  CCHK(check_dims(batch, nf, H, W));
  if (!f || !omega || !feat) return cfail(MFWH_EINVAL, "null array");
  const Net n = make_net(batch, nf, H, W);
  Buf b;
  CCHK(ws_check(n, ws, ws_bytes, &b));
  hipStream_t s = (hipStream_t)stream;
  k_maxabs<<<batch * nf, 256, 0, s>>>(f, (long long)H * W, b.fmax);
  CHIP(hipGetLastError());
  k_features<<<grid_for((long long)batch * H * W * 6 * nf), 256, 0, s>>>(f, b.fmax, omega, batch,
                                                                         nf, H, W, ly, lx, feat);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int mfwh_cnn_scale(int dir, int batch, int nf, int H, int W, float* out, double* v,
                   const double* f, const double* omega, void* ws, size_t ws_bytes,
                   void* stream) {
  CCHK(check_dims(batch, nf, H, W));
  if (!out || !v || !f || !omega || (dir != 0 && dir != 1))
    return cfail(MFWH_EINVAL, "bad scale arguments");
  const Net n = make_net(batch, nf, H, W);
  Buf b;
  CCHK(ws_check(n, ws, ws_bytes, &b));
  hipStream_t s = (hipStream_t)stream;
  k_maxabs<<<batch * nf, 256, 0, s>>>(f, (long long)H * W, b.fmax);
  CHIP(hipGetLastError());
  k_scale<<<grid_for((long long)batch * nf * H * W), 256, 0, s>>>(dir, out, v, b.fmax, omega,
                                                                  batch, nf, H, W);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int mfwh_cnn_normalize(int batch, long long per_sample, float* t, void* stream) {
  if (batch < 1 || per_sample < 1 || !t) return cfail(MFWH_EINVAL, "bad normalize args");
  k_normalize<<<batch, 256, 0, (hipStream_t)stream>>>(t, per_sample);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int mfwh_cnn_forward(int batch, int nf, int H, int W, const float* params, const float* feat,
                     float* out, void* ws, size_t ws_bytes, void* stream) {
  CCHK(check_dims(batch, nf, H, W));
  if (!params || !feat || !out) return cfail(MFWH_EINVAL, "null array");
  const Net n = make_net(batch, nf, H, W);
  Buf b;
  CCHK(ws_check(n, ws, ws_bytes, &b));
  hipStream_t s = (hipStream_t)stream;
  CCHK(forward(n, b, params, feat, s));
  CHIP(hipMemcpyAsync(out, b.a[kLayers - 1], (size_t)n.L[kLayers - 1].P * nf * 4,
                      hipMemcpyDeviceToDevice, s));
  return MFWH_OK;
}

int mfwh_cnn_loss_grad(int batch, int nf, int H, int W, const float* params, const float* feat,
                       const float* target, float* grad, double* loss, void* ws, size_t ws_bytes,
                       void* stream) {
  CCHK(check_dims(batch, nf, H, W));
  if (!params || !feat || !target || !grad) return cfail(MFWH_EINVAL, "null array");
  const Net n = make_net(batch, nf, H, W);
  Buf b;
  CCHK(ws_check(n, ws, ws_bytes, &b));
  hipStream_t s = (hipStream_t)stream;
  CCHK(forward(n, b, params, feat, s));
  const Layer* L = n.L;
  const long long P1 = L[0].P, P2 = L[1].P;
  const long long ny = P1 * nf;
  const int nb = (int)std::min<long long>(kMsePart, (ny + 255) / 256);
  k_mse<<<nb, 256, 0, s>>>(b.a[5], target, ny, b.dy, b.mse);
  CHIP(hipGetLastError());
  // layer 6 (linear)
  CCHK(relu_bwd(b, b.dy, nullptr, P1, nf, 0, s));
  CCHK(layer_wgrad(n, b, 5, b.a[4], grad, s));
  CCHK(layer_dgrad(n, b, 5, b.gD, s));                        // d a5
  CHIP(hipMemcpyAsync(b.s1, b.gD, P1 * kC1 * 4, hipMemcpyDeviceToDevice, s));
  // layer 5: a5 = relu(z5) + a1, input up2(a4)
  CCHK(relu_bwd(b, b.gD, b.z[4], P1, kC1, 1, s));
  CCHK(layer_wgrad(n, b, 4, b.a[3], grad, s));
  CCHK(layer_dgrad(n, b, 4, b.gU, s));                        // d up2(a4), H x W x 64
  k_up2_bwd<<<grid_for(P2 * kC2), 256, 0, s>>>(b.gU, batch, H, W, kC2, n.H2, n.W2, b.gD);
  CHIP(hipGetLastError());                                    // d a4
  CHIP(hipMemcpyAsync(b.s2, b.gD, P2 * kC2 * 4, hipMemcpyDeviceToDevice, s));
  // layer 4: a4 = relu(z4) + a2, input up2(a3)
  CCHK(relu_bwd(b, b.gD, b.z[3], P2, kC2, 1, s));
  CCHK(layer_wgrad(n, b, 3, b.a[2], grad, s));
  CCHK(layer_dgrad(n, b, 3, b.gU, s));                        // d up2(a3), H2 x W2 x 64
  k_up2_bwd<<<grid_for(L[2].P * kC2), 256, 0, s>>>(b.gU, batch, n.H2, n.W2, kC2, n.H3, n.W3, b.gD);
  CHIP(hipGetLastError());                                    // d a3
  // layer 3 (stride 2)
  CCHK(relu_bwd(b, b.gD, b.z[2], L[2].P, kC2, 1, s));
  CCHK(layer_wgrad(n, b, 2, b.a[1], grad, s));
  CCHK(layer_dgrad(n, b, 2, b.gD, s));                        // d a2 (through layer 3)
  k_add<<<grid_for(P2 * kC2), 256, 0, s>>>(b.gD, b.s2, P2 * kC2);
  CHIP(hipGetLastError());
  // layer 2 (stride 2)
  CCHK(relu_bwd(b, b.gD, b.z[1], P2, kC2, 1, s));
  CCHK(layer_wgrad(n, b, 1, b.a[0], grad, s));
  CCHK(layer_dgrad(n, b, 1, b.gU, s));                        // d a1 (through layer 2)
  k_add<<<grid_for(P1 * kC1), 256, 0, s>>>(b.gU, b.s1, P1 * kC1);
  CHIP(hipGetLastError());
  // layer 1
  CCHK(relu_bwd(b, b.gU, b.z[0], P1, kC1, 1, s));
  CCHK(layer_wgrad(n, b, 0, feat, grad, s));
  if (loss) {
    std::vector<double> part(nb);
    CHIP(hipMemcpyAsync(part.data(), b.mse, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    CHIP(hipStreamSynchronize(s));
    double sum = 0.0;
    for (double x : part) sum += x;
    *loss = sum / (double)ny;
  }
  return MFWH_OK;
}

int mfwh_cnn_adam(long long n, float* params, const float* grad, float* m, float* v, int step,
                  float lr, void* stream) {
  if (n < 1 || !params || !grad || !m || !v || step < 1) return cfail(MFWH_EINVAL, "bad adam args");
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
  k_adam<<<grid_for(n), 256, 0, (hipStream_t)stream>>>(params, grad, m, v, n, lr, b1, b2, 1e-8f,
                                                      c1, c2);
  CHIP(hipGetLastError());
  return MFWH_OK;
}

int mfwh_gemm_bf16(int atrans, const void* A, const void* B, float* C, long long M, int N,
                   long long K, int lda, int ldb, int ldc, float* part, void* stream) {
  if (!A || !B || !C || M < 1 || N < 1 || K < 1) return cfail(MFWH_EINVAL, "bad gemm args");
  return gemm(atrans != 0, (const bf16raw*)A, (const bf16raw*)B, C, M, N, K, lda, ldb, ldc, part,
              (hipStream_t)stream);
}

}  // extern "C"
