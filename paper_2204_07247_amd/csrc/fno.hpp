// FP32 Fourier neural operator for the learned warm start of the PAGD solve:
// forward, backward (mean squared error) and Adam, written as HIP kernels.
//
// Network (width W, retained modes M per axis, L spectral layers) on fields
// [B][C][Ny][Nx] (2D) or [B][C][Nz][Ny][Nx] (3D):
//   v0 = P^T x + pb                          (lift, 2 -> W channels)
//   z_l = K_l v_l + W_l^T v_l + b_l,  v_{l+1} = gelu(z_l)  (last layer: no gelu)
//   y = Q^T v_L + qb                         (projection, W -> 1)
// K_l keeps kx in [0, M) and, on y (and z), k in {0..M-1} U {N-M..N-1} of
// the real transform and mixes channels per mode with complex weights
// R_l[i][o][mode].  The truncated transforms are dense products with DFT
// matrices (M << N), so every step of the layer and of its adjoint is one
// strided batched complex GEMM (k_gemm): x, then y per (b, c, z), then z per
// (b, c), and back in reverse order.
//
// Flat parameter layout (shared with the float64 reference of the tests):
// P[2][W], pb[W], per layer R[W][W][modes][re,im] with modes [2M][M] (2D)
// or [2M][2M][M] (3D, kz, ky, kx), Wl[W][W], bl[W]; Q[W], qb.
#pragma once
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

namespace pfch {

struct GemmP {
  int M, N, K;
  const float* A;
  long long sAz, sAm, sAk;  // strides in elements (a complex element is two floats)
  const float* B;
  long long sBz, sBk, sBn;
  float* C;
  long long sCz, sCm, sCn;
  int accumulate;  // 1: C += A B
  // real C only: C[m][n] += bias[m] after the product, and vout (laid out
  // like C) = gelu(C) (act = 1) or C (act = 0); null bias: no epilogue
  const float* bias = nullptr;
  float* vout = nullptr;
  int act = 0;
};

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct f2 {
  float x, y;
};

// Complex multiply-accumulate with operands known real at compile time.
template <bool AC, bool BC>
__device__ __forceinline__ void cmac(f2& c, const f2 a, const f2 b) {
  c.x += a.x * b.x;
  if (AC && BC) c.x -= a.y * b.y;
  if (BC) c.y += a.x * b.y;
  if (AC) c.y += a.y * b.x;
}

// C[z] (+)= A[z] B[z] for z = blockIdx.z.  AC / BC: operand is complex (else
// real); CJA / CJB: conjugate it; CC: C is complex (else the real part is
// stored).  16 x 16 threads, BM x BN output tile (thread (tx, ty) owns rows
// ty + 16 i and columns tx + 16 j), K staged through LDS in steps of 16.
template <bool AC, bool BC, bool CJA, bool CJB, bool CC, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm(GemmP p) {
  constexpr int RM = BM / 16, RN = BN / 16;
  __shared__ f2 As[BM][17];
  __shared__ f2 Bs[16][BN + 1];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const long long m0 = (long long)blockIdx.y * BM, n0 = (long long)blockIdx.x * BN;
  const long long z = blockIdx.z;
  const float* A = p.A + (AC ? 2 : 1) * z * p.sAz;
  const float* B = p.B + (BC ? 2 : 1) * z * p.sBz;
  float* C = p.C + (CC ? 2 : 1) * z * p.sCz;
  f2 acc[RM][RN];
#pragma unroll
  for (int i = 0; i < RM; ++i)
#pragma unroll
    for (int j = 0; j < RN; ++j) acc[i][j] = f2{0.f, 0.f};
  for (int k0 = 0; k0 < p.K; k0 += 16) {
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int e = threadIdx.x + 256 * r;
      const int mm = e >> 4, kk = e & 15;
      const long long m = m0 + mm;
      const int k = k0 + kk;
      f2 a = {0.f, 0.f};
      if (m < p.M && k < p.K) {
        const long long o = m * p.sAm + k * p.sAk;
        if (AC) {
          a.x = A[2 * o];
          a.y = CJA ? -A[2 * o + 1] : A[2 * o + 1];
        } else {
          a.x = A[o];
        }
      }
      As[mm][kk] = a;
    }
#pragma unroll
    for (int r = 0; r < RN; ++r) {
      const int e = threadIdx.x + 256 * r;
      const int kk = e / BN, nn = e % BN;
      const int k = k0 + kk;
      const long long n = n0 + nn;
      f2 b = {0.f, 0.f};
      if (k < p.K && n < p.N) {
        const long long o = k * p.sBk + n * p.sBn;
        if (BC) {
          b.x = B[2 * o];
          b.y = CJB ? -B[2 * o + 1] : B[2 * o + 1];
        } else {
          b.x = B[o];
        }
      }
      Bs[kk][nn] = b;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      f2 bv[RN];
#pragma unroll
      for (int j = 0; j < RN; ++j) bv[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < RM; ++i) {
        const f2 a = As[ty + 16 * i][kk];
#pragma unroll
        for (int j = 0; j < RN; ++j) cmac<AC, BC>(acc[i][j], a, bv[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RM; ++i) {
    const long long m = m0 + ty + 16 * i;
    if (m >= p.M) continue;
#pragma unroll
    for (int j = 0; j < RN; ++j) {
      const long long n = n0 + tx + 16 * j;
      if (n >= p.N) continue;
      const long long o = m * p.sCm + n * p.sCn;
      if (CC) {
        if (p.accumulate) {
          C[2 * o] += acc[i][j].x;
          C[2 * o + 1] += acc[i][j].y;
        } else {
          C[2 * o] = acc[i][j].x;
          C[2 * o + 1] = acc[i][j].y;
        }
      } else {
        float val = p.accumulate ? C[o] + acc[i][j].x : acc[i][j].x;
        if (p.bias) {
          val += p.bias[m];
          if (p.vout) p.vout[z * p.sCz + o] = p.act ? gelu_f(val) : val;
        }
        C[o] = val;
      }
    }
  }
}

__global__ void k_gelu_bwd(const float* __restrict__ dv, const float* __restrict__ z, float* __restrict__ dz,
                           long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  dz[i] = dv[i] * gelu_grad_f(z[i]);
}

// dy = 2 (y - t) / n; part[block] = sum of (y - t)^2 over the block.
__global__ __launch_bounds__(256) void k_mse(const float* __restrict__ y, const float* __restrict__ t,
                                             float* __restrict__ dy, long long n, float* __restrict__ part) {
  __shared__ float red[256];
  float s = 0.f;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const float d = y[i] - t[i];
    dy[i] = 2.0f * d / (float)n;
    s += d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// dv[b][i][p] = Q[i] dy[b][p]
__global__ void k_outer(const float* __restrict__ Q, const float* __restrict__ dy, float* __restrict__ dv,
                        int W, long long P, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const long long p = e % P;
  const int i = (int)((e / P) % W);
  const long long b = e / (P * W);
  dv[e] = Q[i] * dy[b * P + p];
}

__global__ void k_adam(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, long long n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

// Weight and bias gradients of a 1x1 convolution out = sum_i Wt[i][j] X[i] + b[j]
// with upstream gradient Y: part[blk][i][j] = sum over the block's points of
// X[b][i][p] Y[b][j][p] for i < CX, and row CX = sum of Y[b][j][p] (bias).
// Points are the flat (b, p) index space in tiles of 64; block blk takes tiles
// blk, blk + gridDim.x, ... (fixed assignment, so the result is reproducible).
constexpr int WG_TILE = 64, WG_MAXC = 64, WG_MAXACC = 17;
__global__ __launch_bounds__(256) void k_wgrad(const float* __restrict__ X, int CX, const float* __restrict__ Y,
                                               int CY, long long P, long long total, float* __restrict__ part) {
  __shared__ float Xs[WG_MAXC][WG_TILE + 1];
  __shared__ float Ys[WG_MAXC][WG_TILE + 1];
  const int nout = (CX + 1) * CY;
  float acc[WG_MAXACC];
#pragma unroll
  for (int k = 0; k < WG_MAXACC; ++k) acc[k] = 0.f;
  const long long ntiles = (total + WG_TILE - 1) / WG_TILE;
  for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const long long f0 = tile * WG_TILE;
    for (int e = threadIdx.x; e < CX * WG_TILE; e += blockDim.x) {
      const int i = e / WG_TILE, t = e % WG_TILE;
      const long long f = f0 + t;
      float v = 0.f;
      if (f < total) {
        const long long b = f / P, p = f % P;
        v = X[(b * CX + i) * P + p];
      }
      Xs[i][t] = v;
    }
    for (int e = threadIdx.x; e < CY * WG_TILE; e += blockDim.x) {
      const int j = e / WG_TILE, t = e % WG_TILE;
      const long long f = f0 + t;
      float v = 0.f;
      if (f < total) {
        const long long b = f / P, p = f % P;
        v = Y[(b * CY + j) * P + p];
      }
      Ys[j][t] = v;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < WG_MAXACC; ++k) {
      const int o = threadIdx.x + 256 * k;
      if (o < nout) {
        const int i = o / CY, j = o % CY;
        float s = 0.f;
        if (i < CX) {
          for (int t = 0; t < WG_TILE; ++t) s += Xs[i][t] * Ys[j][t];
        } else {
          for (int t = 0; t < WG_TILE; ++t) s += Ys[j][t];
        }
        acc[k] += s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < WG_MAXACC; ++k) {
    const int o = threadIdx.x + 256 * k;
    if (o < nout) part[(long long)blockIdx.x * nout + o] = acc[k];
  }
}

// Sum the per-block partials of k_wgrad: out_w[i][j] for i < CX, out_b[j]
// for the bias row.  Blocks of 64 x 16 threads: each of the 16 slices sums
// the partials k = slice (mod 16) in order, then the slices are added in
// order (a fixed order, independent of timing).
constexpr int WG_RED_SLICES = 16;
__global__ __launch_bounds__(64 * WG_RED_SLICES) void k_wgrad_reduce(const float* __restrict__ part, int nblk,
                                                                     int CX, int CY, float* __restrict__ out_w,
                                                                     float* __restrict__ out_b) {
  __shared__ float red[WG_RED_SLICES][64];
  const int o = blockIdx.x * 64 + threadIdx.x;
  const int nout = (CX + 1) * CY;
  float s = 0.f;
  if (o < nout)
    for (int k = threadIdx.y; k < nblk; k += WG_RED_SLICES) s += part[(long long)k * nout + o];
  red[threadIdx.y][threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.y != 0 || o >= nout) return;
  float t = 0.f;
  for (int q = 0; q < WG_RED_SLICES; ++q) t += red[q][threadIdx.x];
  const int i = o / CY, j = o % CY;
  if (i < CX)
    out_w[o] = t;
  else
    out_b[j] = t;
}

// y[b][p] = sum_i Q[i] v[b][i][p] + qb
__global__ void k_project(const float* __restrict__ v, const float* __restrict__ Q, const float* __restrict__ qb,
                          float* __restrict__ y, int W, long long P, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const long long b = e / P, p = e % P;
  float s = qb[0];
  for (int i = 0; i < W; ++i) s += Q[i] * v[(b * W + i) * P + p];
  y[e] = s;
}

// out = sum of part[0..n) in order (one thread); float partials, double sum.
__global__ void k_sum_parts_f(const float* __restrict__ part, int n, double scale, double* __restrict__ out) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  double s = 0.0;
  for (int k = 0; k < n; ++k) s += (double)part[k];
  *out = s * scale;
}

// ---------------------------------------------------------------------------
// Learned guess kernels.  The reductions run on a fixed grid of GUESS_BLOCKS
// blocks of 256 threads (per-thread sums over a fixed stride, then the
// block's tree), finished by one block in a fixed order, so a batched guess
// equals the instance's solo guess.  Fields are read two points per lane
// (P even: every grid has an even row length).
// ---------------------------------------------------------------------------
constexpr int GUESS_BLOCKS = 1024;

// Tree sum of r[0..256) in LDS; the result is returned to every thread.
__device__ __forceinline__ double guess_tree(double* r, double v) {
  r[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) r[threadIdx.x] += r[threadIdx.x + o];
    __syncthreads();
  }
  const double t = r[0];
  __syncthreads();
  return t;
}

// Network inputs of a learned guess from the step history:
// x[0] = (u^n - mu)/su, x[1] = (u^n - u^{n-1})/sd (as k_fno_inputs).  With
// x0 given (the last step's learned guess e + g c, c its correction kept in
// float) also the per-block partial sums of c (u^n - x0) and c^2, u^n being
// the solution that step reached: gpart[2b], gpart[2b + 1].
__global__ __launch_bounds__(256) void k_guess_inputs(const double* __restrict__ unm1,
                                                      const double* __restrict__ un, long long P, double mu,
                                                      double su, double sd, float* __restrict__ x,
                                                      const double* __restrict__ x0,
                                                      const float* __restrict__ c, double* __restrict__ gpart) {
  __shared__ double r[256];
  const long long h = P >> 1;
  const double2* __restrict__ a2 = reinterpret_cast<const double2*>(un);
  const double2* __restrict__ b2 = reinterpret_cast<const double2*>(unm1);
  float2* __restrict__ xa = reinterpret_cast<float2*>(x);
  float2* __restrict__ xd = reinterpret_cast<float2*>(x + P);
  double s1 = 0.0, s2 = 0.0;
  const long long stride = (long long)GUESS_BLOCKS * 256;
  if (x0) {
    const double2* __restrict__ g2 = reinterpret_cast<const double2*>(x0);
    const float2* __restrict__ c2v = reinterpret_cast<const float2*>(c);
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < h; q += stride) {
      const double2 a = a2[q], b = b2[q], g = g2[q];
      const float2 cv = c2v[q];
      xa[q] = make_float2((float)((a.x - mu) / su), (float)((a.y - mu) / su));
      xd[q] = make_float2((float)((a.x - b.x) / sd), (float)((a.y - b.y) / sd));
      const double c0 = (double)cv.x, c1 = (double)cv.y;
      s1 += c0 * (a.x - g.x);
      s1 += c1 * (a.y - g.y);
      s2 += c0 * c0;
      s2 += c1 * c1;
    }
    const double t1 = guess_tree(r, s1);
    const double t2 = guess_tree(r, s2);
    if (threadIdx.x == 0) {
      gpart[2 * blockIdx.x] = t1;
      gpart[2 * blockIdx.x + 1] = t2;
    }
  } else {
    for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < h; q += stride) {
      const double2 a = a2[q], b = b2[q];
      xa[q] = make_float2((float)((a.x - mu) / su), (float)((a.y - mu) / su));
      xd[q] = make_float2((float)((a.x - b.x) / sd), (float)((a.y - b.y) / sd));
    }
  }
}

// Per-block float64 partial sums of the network output y (float, P points).
__global__ __launch_bounds__(256) void k_guess_ysum(const float* __restrict__ y, long long P,
                                                    double* __restrict__ part) {
  __shared__ double r[256];
  const long long h = P >> 1;
  const float2* __restrict__ y2 = reinterpret_cast<const float2*>(y);
  double s = 0.0;
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < h; q += (long long)GUESS_BLOCKS * 256) {
    const float2 v = y2[q];
    s += (double)v.x;
    s += (double)v.y;
  }
  const double t = guess_tree(r, s);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One block: the mean of y from its partials (ypart[0..GUESS_BLOCKS)) into
// ypart[GUESS_BLOCKS], and the gain of the correction.  Without the last
// step's gain partials the gain is gain_in[0] (the gain the last guess
// used).  With them, the fitted gain is that step's least-squares gain
// gf = g + sum c (x - x0) / sum c^2 clamped to [0, 1] (g the gain the last
// guess used: gf is the gain of the last correction against x - e whatever
// g was), and the gain used is gf if gf >= gate, else 0 (the correction is
// left out).  The gain used goes to gain_out[0]; the fitted gain (or
// gain_in[0]) to gain_pub[0] (pinned host memory, for the statistics and
// the host's gate).
__global__ __launch_bounds__(256) void k_guess_scalars(double* __restrict__ ypart, long long P,
                                                       const double* __restrict__ gain_in,
                                                       const double* __restrict__ gpart, double gate,
                                                       double* __restrict__ gain_out, double* gain_pub) {
  __shared__ double r[256];
  double s = 0.0, s1 = 0.0, s2 = 0.0;
  for (int k = threadIdx.x; k < GUESS_BLOCKS; k += 256) s += ypart[k];
  if (gpart)
    for (int k = threadIdx.x; k < GUESS_BLOCKS; k += 256) {
      s1 += gpart[2 * k];
      s2 += gpart[2 * k + 1];
    }
  const double t = guess_tree(r, s);
  const double t1 = guess_tree(r, s1);
  const double t2 = guess_tree(r, s2);
  if (threadIdx.x == 0) {
    double g = gain_in[0], gf = g;
    if (gpart && t2 > 0.0) {
      gf = fmin(1.0, fmax(0.0, g + t1 / t2));
      g = gf >= gate ? gf : 0.0;
    }
    ypart[GUESS_BLOCKS] = t / (double)P;
    gain_out[0] = g;
    gain_pub[0] = gf;
    __threadfence_system();
  }
}

// Learned initial guess: x0 = u^n + rho (u^n - u^{n-1}) + g c with the
// correction c = so (y - mean(y)), projected to zero mean so that x0 keeps
// the mass of the extrapolation (the solve preserves the mean of its
// initial guess); mean and g from k_guess_scalars.  c is kept (float) in
// c_out for the next step's gain.
__global__ __launch_bounds__(256) void k_learned_guess(const double* __restrict__ un,
                                                       const double* __restrict__ unm1, double rho, double so,
                                                       const float* __restrict__ y,
                                                       const double* __restrict__ mean_p,
                                                       const double* __restrict__ gain_p, long long P,
                                                       double* __restrict__ x0, float* __restrict__ c_out) {
  const double mean = mean_p[0], g = gain_p[0];
  const long long h = P >> 1;
  const double2* __restrict__ a2 = reinterpret_cast<const double2*>(un);
  const double2* __restrict__ b2 = reinterpret_cast<const double2*>(unm1);
  const float2* __restrict__ y2 = reinterpret_cast<const float2*>(y);
  double2* __restrict__ o2 = reinterpret_cast<double2*>(x0);
  float2* __restrict__ c2v = reinterpret_cast<float2*>(c_out);
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < h;
       q += (long long)gridDim.x * blockDim.x) {
    const double2 a = a2[q], b = b2[q];
    const float2 yv = y2[q];
    const double c0 = so * ((double)yv.x - mean), c1 = so * ((double)yv.y - mean);
    o2[q] = make_double2(a.x + rho * (a.x - b.x) + g * c0, a.y + rho * (a.y - b.y) + g * c1);
    c2v[q] = make_float2((float)c0, (float)c1);
  }
}

// Network inputs and (optional) targets from float64 fields:
// x[0] = (u^n - mu)/su, x[1] = (u^n - u^{n-1})/sd,
// t = (u^{n+1} - (u^n + rho (u^n - u^{n-1})))/so.
__global__ void k_fno_inputs(const double* __restrict__ unm1, const double* __restrict__ un,
                             const double* __restrict__ unp1, long long P, double rho, double mu, double su,
                             double sd, double so, float* __restrict__ x, float* __restrict__ t) {
  const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  const double a = un[p], b = unm1[p];
  x[p] = (float)((a - mu) / su);
  x[P + p] = (float)((a - b) / sd);
  if (t) t[p] = (float)((unp1[p] - (a + rho * (a - b))) / so);
}

struct Resampler;

struct Fno {
  int W = 0, M = 0, L = 0, nz = 1, ny = 0, nx = 0, maxb = 0, ndim = 2;
  long long P = 0, n = 0, MM = 0;  // P grid points, MM retained modes (2M^2 or 4M^3)
  hipStream_t s = nullptr;
  float *theta = nullptr, *grad = nullptr, *am = nullptr, *av = nullptr;
  // complex DFT matrices: Fx [Nx][M], Fy [2M][Ny], Fz [2M][Nz] forward;
  // Gz [Nz][2M], Gy [Ny][2M], Gx [M][Nx] inverse (Gx carries 1/P and the
  // weight 2 of the kx > 0 half-spectrum columns)
  float *Fx = nullptr, *Fy = nullptr, *Fz = nullptr, *Gz = nullptr, *Gy = nullptr, *Gx = nullptr;
  std::vector<float*> v, z, vh;  // v[0..L], z[0..L-1], vh[0..L-1]
  // S1 [B][W][Nz][Ny][M] after the x transform, S2 [B][W][Nz][2M][M] after
  // the y transform (3D only), Yb / Yb2 [B][W][modes]
  float *S1 = nullptr, *S2 = nullptr, *Yb = nullptr, *Yb2 = nullptr;
  float *xin = nullptr, *y = nullptr, *dy = nullptr, *dvA = nullptr, *dvB = nullptr;
  float *wpart = nullptr, *lpart = nullptr;
  double *loss = nullptr, *h_loss = nullptr, *ypart = nullptr;
  int wg_blocks = 0;
  std::vector<void*> allocs;
  std::vector<void*> host_allocs;
  long long oP = 0, opb = 0, oQ = 0, oqb = 0;
  std::vector<long long> oR, oW, ob;
  std::vector<Resampler*> rs;  // one per fine grid the network is used on (2D)
  rocblas_handle blas = nullptr;  // the resampling products (made with the first resampler)
};

inline long long fno_modes(long long M, int ndim) { return ndim == 3 ? 4 * M * M * M : 2 * M * M; }

inline long long fno_count(long long W, long long M, long long L, int ndim = 2) {
  return 2 * W + W + L * (W * W * fno_modes(M, ndim) * 2 + W * W + W) + W + 1;
}

constexpr int FNO_LOSS_BLOCKS = 256;

// Launches k_gemm; an M beyond the grid's y extent (65535 tiles) is split
// into row chunks, each a launch on offset A and C.
template <bool AC, bool BC, bool CJA, bool CJB, bool CC, int BM, int BN>
inline hipError_t gemm_launch(const GemmP& p, long long Z, hipStream_t s) {
  const long long gx = (p.N + BN - 1) / BN;
  if (Z > 65535 || gx > 0x7fffffffLL) return hipErrorInvalidConfiguration;
  constexpr long long CHUNK = 65535LL * BM;
  for (long long m0 = 0; m0 < p.M; m0 += CHUNK) {
    GemmP q = p;
    q.M = (int)std::min<long long>(CHUNK, p.M - m0);
    q.A = p.A + (AC ? 2 : 1) * m0 * p.sAm;
    q.C = p.C + (CC ? 2 : 1) * m0 * p.sCm;
    if (p.bias) q.bias = p.bias + m0;
    if (p.vout) q.vout = p.vout + m0 * p.sCm;
    const long long gy = (q.M + BM - 1) / BM;
    hipLaunchKernelGGL((k_gemm<AC, BC, CJA, CJB, CC, BM, BN>), dim3((unsigned)gx, (unsigned)gy, (unsigned)Z),
                       dim3(256), 0, s, q);
  }
  return hipGetLastError();
}

inline GemmP gp_make(long long M, long long N, long long K, const float* A, long long sAz, long long sAm,
                     long long sAk, const float* B, long long sBz, long long sBk, long long sBn, float* C,
                     long long sCz, long long sCm, long long sCn, int acc) {
  GemmP p;
  p.M = (int)M;
  p.N = (int)N;
  p.K = (int)K;
  p.A = A;
  p.sAz = sAz;
  p.sAm = sAm;
  p.sAk = sAk;
  p.B = B;
  p.sBz = sBz;
  p.sBk = sBk;
  p.sBn = sBn;
  p.C = C;
  p.sCz = sCz;
  p.sCm = sCm;
  p.sCn = sCn;
  p.accumulate = acc;
  return p;
}

#define FNO_CHK(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

inline unsigned blocks_for(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------------------
// Band-limited resampling between an instance's grid (Ny x Nx) and the
// coarser grid a network runs on (Ncy x Ncx, the network's own grid).  The
// modes |k| < Nc/2 of each axis are kept (the coarse grid's Nyquist mode is
// dropped, so both directions are real), as products with real matrices:
//   down (fine -> coarse):  c = Dy f Dx,
//     Dx[x][xc] = (1/Nx) (1 + 2 sum_{k=1}^{Ncx/2-1} cos 2 pi k (xc/Ncx - x/Nx)),
//   up (coarse -> fine):    f = Uy c Ux,
//     Ux[xc][x] = (1/Ncx) (1 + 2 sum_{k=1}^{Ncx/2-1} cos 2 pi k (x/Nx - xc/Ncx)),
// and the same on y.  down samples the band-limited part of a fine field at
// the coarse points; up interpolates coarse samples band-limitedly; both
// keep the mean.  Each is two plain float32 matrix products (x, then y),
// done by rocBLAS on the network's stream.
// ---------------------------------------------------------------------------
struct Resampler {
  int ny = 0, nx = 0;             // fine grid
  int nb = 0;                     // samples the buffers below hold (the network's batch)
  float *Dx = nullptr, *Dy = nullptr;  // [Nx][Ncx], [Ncy][Ny]
  float *Uy = nullptr, *Ux = nullptr;  // [Ny][Ncy], [Ncx][Nx]
  float *T1 = nullptr;            // [nb][2][Ny][Ncx]
  float *T2 = nullptr;            // [nb][Ny][Ncx]
  float *Xf = nullptr;            // [nb][2][Ny][Nx] fine network inputs
  float *yf = nullptr;            // [nb][Ny][Nx] fine corrections (or fine targets)
};

// c[b][ch][Ncy][Ncx] = Dy f[b][ch] Dx for nb samples of `ch` fine fields
// f[b][ch][Ny][Nx]: one strided batched product per stage, each sample's
// product of the same shape whatever nb is.
inline hipError_t resample_down(const Fno& F, const Resampler& R, const float* f, int ch, float* c, int nb,
                                hipStream_t s);
// R.yf[b] = Uy c[b] Ux for nb coarse fields c[b] = c + b P (P coarse points).
inline hipError_t resample_up(const Fno& F, const Resampler& R, const float* c, int nb, hipStream_t s);

// Forward pass for `B` samples x[B][2][grid]; keeps every layer's input,
// pre-activation and retained spectrum for the backward pass; y[B][grid].
inline hipError_t fno_forward(Fno& F, const float* x, int B, hipStream_t s) {
  const long long W = F.W, M = F.M, P = F.P, nz = F.nz, ny = F.ny, nx = F.nx, MM = F.MM;
  const long long M2 = 2 * M * M;  // modes of one (b, c, z) after the y transform
  const bool d3 = F.ndim == 3;
  const float* th = F.theta;
  // lift, with its bias in the product's epilogue
  GemmP lift = gp_make(W, P, 2, th + F.oP, 0, 1, W, x, 2 * P, P, 1, F.v[0], W * P, P, 1, 0);
  lift.bias = th + F.opb;
  FNO_CHK((gemm_launch<false, false, false, false, false, 32, 64>(lift, B, s)));
  for (int l = 0; l < F.L; ++l) {
    const float* vin = F.v[l];
    float* yk = d3 ? F.S2 : F.vh[l];  // y-transform output
    // S1 = v Fx over x
    FNO_CHK((gemm_launch<false, true, false, false, true, 64, 16>(
        gp_make(B * W * nz * ny, M, nx, vin, 0, nx, 1, F.Fx, 0, M, 1, F.S1, 0, M, 1, 0), 1, s)));
    // Fy S1 over y (retained ky rows), per (b, c, z)
    FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
        gp_make(2 * M, M, ny, F.Fy, 0, ny, 1, F.S1, ny * M, M, 1, yk, M2, M, 1, 0), B * W * nz, s)));
    // 3D: vh = Fz S2 over z (retained kz rows), per (b, c)
    if (d3)
      FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
          gp_make(2 * M, M2, nz, F.Fz, 0, nz, 1, F.S2, nz * M2, M2, 1, F.vh[l], MM, M2, 1, 0), B * W, s)));
    // per-mode channel mixing Y[b][o] = sum_i vh[b][i] R[i][o]
    FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
        gp_make(B, W, W, F.vh[l], 1, W * MM, MM, th + F.oR[l], 1, W * MM, MM, F.Yb, 1, W * MM, MM, 0), MM, s)));
    // 3D: S2 = Gz Y over z
    if (d3)
      FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
          gp_make(nz, M2, 2 * M, F.Gz, 0, 2 * M, 1, F.Yb, MM, M2, 1, F.S2, nz * M2, M2, 1, 0), B * W, s)));
    // S1 = Gy (Y or S2) over y
    FNO_CHK((gemm_launch<true, true, false, false, true, 64, 16>(
        gp_make(ny, M, 2 * M, F.Gy, 0, 2 * M, 1, d3 ? F.S2 : F.Yb, M2, M, 1, F.S1, ny * M, M, 1, 0), B * W * nz,
        s)));
    // z = Re(S1 Gx) over x
    FNO_CHK((gemm_launch<true, true, false, false, false, 32, 64>(
        gp_make(B * W * nz * ny, nx, M, F.S1, 0, M, 1, F.Gx, 0, nx, 1, F.z[l], 0, nx, 1, 0), 1, s)));
    // z += W_l^T v + b_l and v_{l+1} = gelu(z) (z for the last layer), in
    // the product's epilogue
    GemmP cv = gp_make(W, P, W, th + F.oW[l], 0, 1, W, vin, W * P, P, 1, F.z[l], W * P, P, 1, 1);
    cv.bias = th + F.ob[l];
    cv.vout = F.v[l + 1];
    cv.act = l < F.L - 1 ? 1 : 0;
    FNO_CHK((gemm_launch<false, false, false, false, false, 32, 64>(cv, B, s)));
  }
  hipLaunchKernelGGL(k_project, dim3(blocks_for(B * P)), dim3(256), 0, s, (const float*)F.v[F.L], th + F.oQ,
                     th + F.oqb, F.y, (int)W, P, B * P);
  return hipGetLastError();
}

inline hipError_t wgrad(Fno& F, const float* X, int CX, const float* Y, int CY, long long total, float* out_w,
                        float* out_b, hipStream_t s) {
  hipLaunchKernelGGL(k_wgrad, dim3(F.wg_blocks), dim3(256), 0, s, X, CX, Y, CY, F.P, total, F.wpart);
  const int nout = (CX + 1) * CY;
  hipLaunchKernelGGL(k_wgrad_reduce, dim3((nout + 63) / 64), dim3(64, WG_RED_SLICES), 0, s, (const float*)F.wpart,
                     F.wg_blocks, CX, CY, out_w, out_b);
  return hipGetLastError();
}

// Forward, mean squared error against t[B][grid] and the gradient of the
// loss with respect to every parameter (into F.grad).  F.loss receives the
// loss (device float64).  The complex adjoints carry the conjugate of the
// gradient, so every transform's adjoint is its plain transpose.
inline hipError_t fno_backward(Fno& F, const float* x, const float* t, int B, hipStream_t s) {
  FNO_CHK(fno_forward(F, x, B, s));
  const long long W = F.W, M = F.M, P = F.P, nz = F.nz, ny = F.ny, nx = F.nx, MM = F.MM;
  const long long M2 = 2 * M * M;
  const bool d3 = F.ndim == 3;
  const long long nB = (long long)B * P;
  const float* th = F.theta;
  float* g = F.grad;
  hipLaunchKernelGGL(k_mse, dim3(FNO_LOSS_BLOCKS), dim3(256), 0, s, (const float*)F.y, t, F.dy, nB, F.lpart);
  hipLaunchKernelGGL(k_sum_parts_f, dim3(1), dim3(1), 0, s, (const float*)F.lpart, FNO_LOSS_BLOCKS,
                     1.0 / (double)nB, F.loss);
  FNO_CHK(wgrad(F, F.v[F.L], (int)W, F.dy, 1, nB, g + F.oQ, g + F.oqb, s));
  float* dv = F.dvA;
  float* dvin = F.dvB;
  hipLaunchKernelGGL(k_outer, dim3(blocks_for(B * W * P)), dim3(256), 0, s, th + F.oQ, (const float*)F.dy, dv,
                     (int)W, P, B * W * P);
  for (int l = F.L - 1; l >= 0; --l) {
    if (l < F.L - 1)
      hipLaunchKernelGGL(k_gelu_bwd, dim3(blocks_for(B * W * P)), dim3(256), 0, s, (const float*)dv,
                         (const float*)F.z[l], dv, B * W * P);
    const float* dz = dv;
    const float* vin = F.v[l];
    float* yk = d3 ? F.S2 : F.Yb;  // adjoint of the y transform, per (b, c, z)
    FNO_CHK(wgrad(F, vin, (int)W, dz, (int)W, nB, g + F.oW[l], g + F.ob[l], s));
    // dvin = W_l dz
    FNO_CHK((gemm_launch<false, false, false, false, false, 32, 64>(
        gp_make(W, P, W, th + F.oW[l], 0, W, 1, dz, W * P, P, 1, dvin, W * P, P, 1, 0), B, s)));
    // D_S1 = dz Gx^T
    FNO_CHK((gemm_launch<false, true, false, false, true, 64, 16>(
        gp_make(B * W * nz * ny, M, nx, dz, 0, nx, 1, F.Gx, 0, 1, nx, F.S1, 0, M, 1, 0), 1, s)));
    // Gy^T D_S1
    FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
        gp_make(2 * M, M, ny, F.Gy, 0, 1, 2 * M, F.S1, ny * M, M, 1, yk, M2, M, 1, 0), B * W * nz, s)));
    // 3D: D_Y = Gz^T D_S2
    if (d3)
      FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
          gp_make(2 * M, M2, nz, F.Gz, 0, 1, 2 * M, F.S2, nz * M2, M2, 1, F.Yb, MM, M2, 1, 0), B * W, s)));
    // grad R = conj(sum_b vh[b][i] D_Y[b][o]) per mode, stored (re, im)
    FNO_CHK((gemm_launch<true, true, true, true, true, 32, 32>(
        gp_make(W, W, B, F.vh[l], 1, MM, W * MM, F.Yb, 1, W * MM, MM, g + F.oR[l], 1, W * MM, MM, 0), MM, s)));
    // D_vh[b][i] = sum_o D_Y[b][o] R[i][o]
    FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
        gp_make(B, W, W, F.Yb, 1, W * MM, MM, th + F.oR[l], 1, MM, W * MM, F.Yb2, 1, W * MM, MM, 0), MM, s)));
    // 3D: D_S2 = Fz^T D_vh
    if (d3)
      FNO_CHK((gemm_launch<true, true, false, false, true, 32, 32>(
          gp_make(nz, M2, 2 * M, F.Fz, 0, 1, nz, F.Yb2, MM, M2, 1, F.S2, nz * M2, M2, 1, 0), B * W, s)));
    // D_S1 = Fy^T (D_vh or D_S2)
    FNO_CHK((gemm_launch<true, true, false, false, true, 64, 16>(
        gp_make(ny, M, 2 * M, F.Fy, 0, 1, ny, d3 ? F.S2 : F.Yb2, M2, M, 1, F.S1, ny * M, M, 1, 0), B * W * nz,
        s)));
    // dvin += Re(D_S1 Fx^T)
    FNO_CHK((gemm_launch<true, true, false, false, false, 32, 64>(
        gp_make(B * W * nz * ny, nx, M, F.S1, 0, M, 1, F.Fx, 0, 1, M, dvin, 0, nx, 1, 1), 1, s)));
    float* tmp = dv;
    dv = dvin;
    dvin = tmp;
  }
  FNO_CHK(wgrad(F, x, 2, dv, (int)W, nB, g + F.oP, g + F.opb, s));
  return hipGetLastError();
}

// Row-major C[M][N] = A[M][K] B[K][N] (lda = K, ldb = N, ldc = N), `batch`
// products with strides sA, sB, sC: column-major rocBLAS computes C^T = B^T A^T.
inline hipError_t sgemm_rm(const Fno& F, int M, int N, int K, const float* A, long long sA, const float* B,
                           long long sB, float* C, long long sC, int batch, hipStream_t s) {
  const float one = 1.0f, zero = 0.0f;
  if (rocblas_set_stream(F.blas, s) != rocblas_status_success) return hipErrorUnknown;
  const rocblas_status st = rocblas_sgemm_strided_batched(F.blas, rocblas_operation_none, rocblas_operation_none, N, M,
                                                          K, &one, B, N, sB, A, K, sA, &zero, C, N, sC, batch);
  return st == rocblas_status_success ? hipSuccess : hipErrorUnknown;
}

inline hipError_t resample_down(const Fno& F, const Resampler& R, const float* f, int ch, float* c, int nb,
                                hipStream_t s) {
  const long long ny = R.ny, nx = R.nx, ncy = F.ny, ncx = F.nx;
  // T1[b][ch * Ny + y][xc] = sum_x f[b][ch][y][x] Dx[x][xc]
  FNO_CHK(sgemm_rm(F, (int)(ch * ny), (int)ncx, (int)nx, f, ch * ny * nx, R.Dx, 0, R.T1, ch * ny * ncx, nb, s));
  // c[b][ch][yc][xc] = sum_y Dy[yc][y] T1[b][ch][y][xc]
  FNO_CHK(sgemm_rm(F, (int)ncy, (int)ncx, (int)ny, R.Dy, 0, R.T1, ny * ncx, c, ncy * ncx, nb * ch, s));
  return hipSuccess;
}

inline hipError_t resample_up(const Fno& F, const Resampler& R, const float* c, int nb, hipStream_t s) {
  const long long ny = R.ny, nx = R.nx, ncy = F.ny, ncx = F.nx;
  // T2[b][y][xc] = sum_yc Uy[y][yc] c[b][yc][xc]
  FNO_CHK(sgemm_rm(F, (int)ny, (int)ncx, (int)ncy, R.Uy, 0, c, F.P, R.T2, ny * ncx, nb, s));
  // yf[b][y][x] = sum_xc T2[b][y][xc] Ux[xc][x]
  FNO_CHK(sgemm_rm(F, (int)ny, (int)nx, (int)ncx, R.T2, ny * ncx, R.Ux, 0, R.yf, ny * nx, nb, s));
  return hipSuccess;
}

}  // namespace pfch
