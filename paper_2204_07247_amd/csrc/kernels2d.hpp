// Fused PAGD kernels for 2D PFC / FCH steps on gfx950 (FP64).
//
// One PAGD iteration j (Alg. 2) is two launches:
//   col_iter(j): per column tile of the half spectrum, forward y-FFT of the
//                row-transformed fields, the k-space residual
//                r^ = -[ (a/theta v^ + g^) / (M k^2) + mu^ ]  (eq. obj:G'),
//                the averaged-Newton solve d^ = r^ / L^(k) (Sec. 3.4.1), and
//                the inverse y-FFT of d^ (FCH: also of -k^2 d^).
//   row_iter(j): per row pair, inverse x-FFT giving d_j (and Delta d_j),
//                y_j = x_j + lambda_j (x_j - x_{j-1}),  x_{j+1} = y_j + s d_j,
//                ||d_j||_inf, then already the start of iteration j+1:
//                y_{j+1}, v_breve, the pointwise nonlinear terms and the
//                forward x-FFT of them.
// The iterate lives only in real space (ring x_j at X[j % 3]); k-space
// quantities are recomputed from transforms each iteration, and the step
// constant g = (b - a (1-theta)/theta) u^n + c u^{n-1} is transformed once
// per step (a y + b u^n + c u^{n-1} = (a/theta) v_breve + g).
//
// Row layout: real fields are [rows][nx] (x fastest); spectral rows are
// [field][rows][nh], nh = nx/2 + 1, complex FP64.
#pragma once
#include "fft.hpp"
#include "pfch_dev.hpp"

namespace pfch {

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

// True when iteration j must not run: the cap is reached, or iteration j-1
// met the tolerance or produced a non-finite norm.  Iterations that were
// skipped leave their norm slot at 0, which also reads as "stopped".
__device__ __forceinline__ bool stopped_before(const InstDev* I, int j) {
  if (j >= I->max_iter) return true;
  if (j == 0) return false;
  const uint64_t b = I->norms[j - 1];
  return b < I->tol_bits || b >= INF_BITS;
}

// Number of active lanes in this thread's wave (blocks may be smaller than
// a wave on tiny grids).
__device__ __forceinline__ int wave_width() {
  const int rem = (int)blockDim.x - (int)(threadIdx.x & ~63u);
  return rem < 64 ? rem : 64;
}

// Deterministic block sum (fixed shuffle tree, then waves in order).  The
// result is valid in thread 0.  `red` holds one double per wave.
__device__ __forceinline__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, width = wave_width();
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double o = __shfl_xor(v, off, 64);
    if ((lane ^ off) < width) v += o;
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) s += red[w];
  }
  return s;
}

__device__ __forceinline__ uint64_t block_max_bits(uint64_t v, uint64_t* red) {
  const int lane = threadIdx.x & 63, width = wave_width();
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint64_t o = (uint64_t)__shfl_xor((long long)v, off, 64);
    if ((lane ^ off) < width && o > v) v = o;
  }
  const int wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  uint64_t m = 0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int w = 0; w < nw; ++w) m = red[w] > m ? red[w] : m;
  }
  return m;
}

// Z[k] = A[k] + i B[k] over the full length from two Hermitian half spectra.
template <class P>
__device__ __forceinline__ void load_pack(c2 (&v)[P::RMAX], const c2* __restrict__ A,
                                          const c2* __restrict__ B, int t) {
  constexpr int N = P::N, T = P::T;
#pragma unroll
  for (int m = 0; m < P::RMAX; ++m) {
    const int k = t + m * T;
    const bool hi = k > N / 2;
    const int kk = hi ? N - k : k;
    c2 a = A[kk], b = B[kk];
    if (hi) {
      a.y = -a.y;
      b.y = -b.y;
    }
    v[m] = c2{a.x - b.y, a.y + b.x};
  }
}

// After the forward transform of Z = a + i b (a, b real): store the half
// spectra A[k] = (Z[k] + conj Z[N-k]) / 2 and B[k] = -i (Z[k] - conj Z[N-k]) / 2.
template <class P>
__device__ __forceinline__ void unpack_store(const c2 (&v)[P::RMAX], c2* lds, c2* __restrict__ A,
                                             c2* __restrict__ B, int t) {
  constexpr int N = P::N, T = P::T;
#pragma unroll
  for (int m = 0; m < P::RMAX; ++m) lds[lds_idx(t + m * T)] = v[m];
  __syncthreads();
#pragma unroll
  for (int m = 0; m <= P::RMAX / 2; ++m) {
    const int k = t + m * T;
    if (k <= N / 2) {
      const c2 z = lds[lds_idx(k)];
      const c2 w = lds[lds_idx(k == 0 ? 0 : N - k)];
      // conj(w) = (w.x, -w.y)
      A[k] = c2{0.5 * (z.x + w.x), 0.5 * (z.y - w.y)};
      const double dx = z.x - w.x, dy = z.y + w.y;  // z - conj(w)
      B[k] = c2{0.5 * dy, -0.5 * dx};
    }
  }
  __syncthreads();
}

// |k|^2 for column kx and row index ky of a 2D half spectrum.
__device__ __forceinline__ double wavenum2(const InstDev* I, int kx, int ky, int ny) {
  const int kyp = ky <= ny / 2 ? ky : ky - ny;
  const double ax = kx * I->kx_scale, ay = kyp * I->ky_scale;
  return ax * ax + ay * ay;
}

// Averaged-Newton constants (beta_-2, beta_0, beta_2, beta_4) from the setup
// partial sums, summed in a fixed order so every block gets the same values.
__device__ __forceinline__ void betas(const InstDev* I, double& bm2, double& b0, double& b2,
                                      double& b4) {
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < I->nparts; ++i) {
    s0 += I->part[2 * i];
    s1 += I->part[2 * i + 1];
  }
  bm2 = I->a / I->mobility;
  if (I->model == MODEL_PFC) {
    b0 = fabs(s0 * I->inv_p);
    b2 = -2.0;
    b4 = 1.0;
  } else {
    const double e2 = I->eps * I->eps;
    b0 = fabs(s0 * I->inv_p);
    b2 = fabs(s1 * I->inv_p);
    b4 = e2 * e2;
  }
}

// ---------------------------------------------------------------------------
// Column kernel of one PAGD iteration.
// ---------------------------------------------------------------------------
template <class PY, int MODEL>
__global__ __launch_bounds__(256) void k_col_iter(const InstDev* __restrict__ I, int l) {
  extern __shared__ c2 smem[];
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int cb = blockDim.x / T;
  const int c = threadIdx.x % cb, t = threadIdx.x / cb;
  const int nh = I->nh;
  const int kx = blockIdx.x * cb + c;
  const bool valid = kx < nh;
  const int kxc = valid ? kx : nh - 1;
  c2* lds = smem + c * lds_len(N);
  const int64_t fs = I->field_stride;
  c2* __restrict__ S = I->S;

  double bm2, b0, b2, b4;
  betas(I, bm2, b0, b2, b4);
  const double thl = I->theta_l, inv_m = 1.0 / I->mobility, aot = I->a_over_theta;
  const double inv_p = I->inv_p;

  c2 v[RM], acc[RM];
  int bad = 0;
  if constexpr (MODEL == MODEL_PFC) {
    // field 0: N^ = FFT(v_breve^3); field 1: v_breve^
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = S[(int64_t)(t + m * T) * nh + kxc];
    fft<PY, false>(v, lds, I->tw_y, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = v[m];
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = S[fs + (int64_t)(t + m * T) * nh + kxc];
    fft<PY, false>(v, lds, I->tw_y, t);
    const double e1 = 1.0 - I->eps;
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int ky = t + m * T;
      const double k2 = wavenum2(I, kxc, ky, N);
      c2 d = {0.0, 0.0};
      if (k2 > 0.0) {
        const c2 g = I->ghat[(int64_t)ky * nh + kxc];
        const double lin = e1 - 2.0 * k2 + k2 * k2;
        const double ik2 = inv_m / k2;
        // G'^ = (a/theta v^ + g^)/(M k^2) + N^ + lin v^ ; r^ = -G'^
        const double gx = (aot * v[m].x + g.x) * ik2 + acc[m].x + lin * v[m].x;
        const double gy = (aot * v[m].y + g.y) * ik2 + acc[m].y + lin * v[m].y;
        const double L = bm2 / k2 + thl * (b0 + b2 * k2 + b4 * k2 * k2);
        bad |= !(L > 0.0);
        const double sc = -inv_p / L;
        d = c2{gx * sc, gy * sc};
      }
      v[m] = d;
    }
    fft<PY, true>(v, lds, I->tw_y, t);
    if (valid) {
#pragma unroll
      for (int m = 0; m < RM; ++m) S[(int64_t)(t + m * T) * nh + kx] = v[m];
    }
  } else {
    // fields: 0 F'^, 1 p^, 2 v_breve^
    const double e2 = I->eps * I->eps, e4 = e2 * e2, e2h1 = e2 * I->eta1;
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = S[(int64_t)(t + m * T) * nh + kxc];
    fft<PY, false>(v, lds, I->tw_y, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const double k2 = wavenum2(I, kxc, t + m * T, N);
      acc[m] = cscale(v[m], e2 * k2);
    }
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = S[fs + (int64_t)(t + m * T) * nh + kxc];
    fft<PY, false>(v, lds, I->tw_y, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = cadd(acc[m], v[m]);
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = S[2 * fs + (int64_t)(t + m * T) * nh + kxc];
    fft<PY, false>(v, lds, I->tw_y, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int ky = t + m * T;
      const double k2 = wavenum2(I, kxc, ky, N);
      c2 d = {0.0, 0.0};
      if (k2 > 0.0) {
        const c2 g = I->ghat[(int64_t)ky * nh + kxc];
        const double lin = e4 * k2 * k2 - e2h1 * k2;
        const double ik2 = inv_m / k2;
        // mu^ = eps^2 k^2 F'^ + p^ + (eps^4 k^4 - eps^2 eta1 k^2) v^
        const double gx = (aot * v[m].x + g.x) * ik2 + acc[m].x + lin * v[m].x;
        const double gy = (aot * v[m].y + g.y) * ik2 + acc[m].y + lin * v[m].y;
        const double L = bm2 / k2 + thl * (b0 + b2 * k2 + b4 * k2 * k2);
        bad |= !(L > 0.0);
        const double sc = -inv_p / L;
        d = c2{gx * sc, gy * sc};
      }
      acc[m] = d;
      v[m] = d;
    }
    fft<PY, true>(v, lds, I->tw_y, t);
    if (valid) {
#pragma unroll
      for (int m = 0; m < RM; ++m) S[(int64_t)(t + m * T) * nh + kx] = v[m];
    }
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const double k2 = wavenum2(I, kxc, t + m * T, N);
      v[m] = cscale(acc[m], -k2);
    }
    fft<PY, true>(v, lds, I->tw_y, t);
    if (valid) {
#pragma unroll
      for (int m = 0; m < RM; ++m) S[fs + (int64_t)(t + m * T) * nh + kx] = v[m];
    }
  }
  if (bad && valid) atomicOr(I->flags, FLAG_PRECOND);
}

// ---------------------------------------------------------------------------
// Row kernel of one PAGD iteration (end of j, start of j+1).
// ---------------------------------------------------------------------------
template <class PX>
__device__ __forceinline__ void pfc_forward_row(const InstDev* I, const double (&vb)[PX::RMAX], c2* lds,
                                                int row, int t) {
  constexpr int RM = PX::RMAX;
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) z[m] = c2{vb[m] * vb[m] * vb[m], vb[m]};
  fft<PX, false>(z, lds, I->tw_x, t);
  const int nh = I->nh;
  unpack_store<PX>(z, lds, I->S + (int64_t)row * nh, I->S + I->field_stride + (int64_t)row * nh, t);
}

// FCH pointwise terms at v_breve with Laplacian lv:
//   F' = (v^2-1)(v+tau), F'' = 3v^2 - 1 + 2 tau v, omega = eps^2 lv - F',
//   p = -F'' omega - eta2 F'.
template <class PX>
__device__ __forceinline__ void fch_forward_row(const InstDev* I, const double (&vb)[PX::RMAX],
                                                const double (&lv)[PX::RMAX], c2* lds, int row, int t) {
  constexpr int RM = PX::RMAX;
  const double e2 = I->eps * I->eps, tau = I->tau, eta2 = I->eta2;
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const double u = vb[m];
    const double f1 = (u * u - 1.0) * (u + tau);
    const double f2 = 3.0 * u * u - 1.0 + 2.0 * tau * u;
    const double om = e2 * lv[m] - f1;
    z[m] = c2{f1, -f2 * om - eta2 * f1};
  }
  fft<PX, false>(z, lds, I->tw_x, t);
  const int nh = I->nh;
  unpack_store<PX>(z, lds, I->S + (int64_t)row * nh, I->S + I->field_stride + (int64_t)row * nh, t);
}

template <class PX>
__device__ __forceinline__ void pair_forward(const InstDev* I, const double (&a)[PX::RMAX],
                                             const double (&b)[PX::RMAX], c2* lds, c2* A, c2* B, int t) {
  constexpr int RM = PX::RMAX;
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) z[m] = c2{a[m], b[m]};
  fft<PX, false>(z, lds, I->tw_x, t);
  unpack_store<PX>(z, lds, A, B, t);
}

template <class PX, int MODEL>
__global__ __launch_bounds__(256) void k_row_iter(const InstDev* __restrict__ I, int l) {
  extern __shared__ c2 smem[];
  __shared__ uint64_t red[4];
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (blockIdx.x * teams + team);
  const int nh = I->nh;
  const int64_t fs = I->field_stride;
  const int ne = I->n_eta;
  const double lam = I->lam[j % ne], lamn = I->lam[(j + 1) % ne];
  const double s = I->s, th = I->theta;
  const bool mp = th != 1.0;
  const double* __restrict__ xj = I->X[j % 3];
  const double* __restrict__ xm = I->X[(j + 2) % 3];
  double* __restrict__ xn = I->X[(j + 1) % 3];
  const double* __restrict__ un = I->un;
  uint64_t dmax = 0;

  if constexpr (MODEL == MODEL_PFC) {
    c2 v[RM];
    load_pack<PX>(v, I->S + (int64_t)r0 * nh, I->S + (int64_t)(r0 + 1) * nh, t);
    fft<PX, true>(v, lds, I->tw_x, t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      double vb[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int64_t idx = (int64_t)(r0 + row) * N + t + m * T;
        const double d = row ? v[m].y : v[m].x;
        const double a = xj[idx], b = xm[idx];
        const double y = a + lam * (a - b);
        const double x1 = y + s * d;
        xn[idx] = x1;
        const uint64_t db = dbits(fabs(d));
        dmax = db > dmax ? db : dmax;
        const double yn = x1 + lamn * (x1 - a);
        vb[m] = mp ? th * yn + (1.0 - th) * un[idx] : yn;
      }
      pfc_forward_row<PX>(I, vb, lds, r0 + row, t);
    }
  } else {
    const double* __restrict__ dxj = I->DX[j % 3];
    const double* __restrict__ dxm = I->DX[(j + 2) % 3];
    double* __restrict__ dxn = I->DX[(j + 1) % 3];
    const double* __restrict__ dun = I->dun;
    double vbs[2][RM];
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      const int r = r0 + row;
      c2 v[RM];
      load_pack<PX>(v, I->S + (int64_t)r * nh, I->S + fs + (int64_t)r * nh, t);
      fft<PX, true>(v, lds, I->tw_x, t);
      double lv[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int64_t idx = (int64_t)r * N + t + m * T;
        const double d = v[m].x, ld = v[m].y;
        const double a = xj[idx], b = xm[idx];
        const double la = dxj[idx], lb = dxm[idx];
        const double y = a + lam * (a - b);
        const double ly = la + lam * (la - lb);
        const double x1 = y + s * d;
        const double lx1 = ly + s * ld;
        xn[idx] = x1;
        dxn[idx] = lx1;
        const uint64_t db = dbits(fabs(d));
        dmax = db > dmax ? db : dmax;
        const double yn = x1 + lamn * (x1 - a);
        const double lyn = lx1 + lamn * (lx1 - la);
        vbs[row][m] = mp ? th * yn + (1.0 - th) * un[idx] : yn;
        lv[m] = mp ? th * lyn + (1.0 - th) * dun[idx] : lyn;
      }
      fch_forward_row<PX>(I, vbs[row], lv, lds, r, t);
    }
    pair_forward<PX>(I, vbs[0], vbs[1], lds, I->S + 2 * fs + (int64_t)r0 * nh,
                     I->S + 2 * fs + (int64_t)(r0 + 1) * nh, t);
  }
  const uint64_t bm = block_max_bits(dmax, red);
  if (threadIdx.x == 0) atomicMax((unsigned long long*)&I->norms[j], (unsigned long long)bm);
}

// ---------------------------------------------------------------------------
// Step setup, row part: initial guess, transform of the step constant g,
// partial sums for the averaged-Newton constants and (PFC) the forward
// transforms that start iteration 0.  Block 0 publishes the per-step scalars.
// ---------------------------------------------------------------------------
struct StepArgs {
  const double* un;
  const double* unm1;  // may equal un on the first step
  const double* xin;   // given initial guess, or null to extrapolate
  double rho;          // extrapolation factor dt_{n+1}/dt_n (0 on the first step)
  double a, theta;
  double gu, gm;       // g = gu u^n + gm u^{n-1}
};

template <class PX, int MODEL>
__global__ __launch_bounds__(256) void k_row_setup(InstDev* __restrict__ I, StepArgs sa) {
  extern __shared__ c2 smem[];
  __shared__ double red[4];
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (blockIdx.x * teams + team);
  const int nh = I->nh;
  const int64_t fs = I->field_stride;
  const double th = sa.theta;
  double* __restrict__ x0a = I->X[0];
  double* __restrict__ x0b = I->X[2];

  if (blockIdx.x == 0 && threadIdx.x == 0) {
    I->a = sa.a;
    I->theta = sa.theta;
    I->a_over_theta = sa.a / sa.theta;
    I->un = sa.un;
    *I->iter_base = 0;
    *I->flags = 0;
    I->rec->stop_iter = -1;
    I->rec->flags = 0;
    I->rec->norm_bits = 0;
  }
  {  // clear the per-iteration norm slots
    const int nthreads = gridDim.x * blockDim.x;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < I->max_iter; i += nthreads) I->norms[i] = 0;
  }

  double s0 = 0.0, s1 = 0.0;
  double x0v[2][RM], gv[2][RM];
  const double eps = I->eps, tau = I->tau, e2 = eps * eps;
#pragma unroll
  for (int row = 0; row < 2; ++row) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int64_t idx = (int64_t)(r0 + row) * N + t + m * T;
      const double u = sa.un[idx], um = sa.unm1[idx];
      const double x0 = sa.xin ? sa.xin[idx] : u + sa.rho * (u - um);
      x0a[idx] = x0;
      x0b[idx] = x0;
      x0v[row][m] = x0;
      gv[row][m] = sa.gu * u + sa.gm * um;
      const double vb = th * x0 + (1.0 - th) * u;
      if constexpr (MODEL == MODEL_PFC) {
        s0 += 3.0 * vb * vb + 1.0 - eps;
      } else {
        const double f1 = (vb * vb - 1.0) * (vb + tau);
        const double f2 = 3.0 * vb * vb - 1.0 + 2.0 * tau * vb;
        const double f3 = 6.0 * vb + 2.0 * tau;
        s0 += f2 * f2 - I->eta2 * f2 + f3 * f1;
        s1 += e2 * f2 - I->eta1 * e2;
      }
    }
  }
  if constexpr (MODEL == MODEL_PFC) {
    pair_forward<PX>(I, gv[0], gv[1], lds, I->G + (int64_t)r0 * nh, I->G + (int64_t)(r0 + 1) * nh, t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      double vb[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const int64_t idx = (int64_t)(r0 + row) * N + t + m * T;
        vb[m] = th * x0v[row][m] + (1.0 - th) * sa.un[idx];
      }
      pfc_forward_row<PX>(I, vb, lds, r0 + row, t);
    }
  } else {
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      const int r = r0 + row;
      pair_forward<PX>(I, gv[row], x0v[row], lds, I->G + (int64_t)r * nh, I->G + fs + (int64_t)r * nh, t);
    }
    if (th != 1.0) {
      double ua[RM], ub[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        ua[m] = sa.un[(int64_t)r0 * N + t + m * T];
        ub[m] = sa.un[(int64_t)(r0 + 1) * N + t + m * T];
      }
      pair_forward<PX>(I, ua, ub, lds, I->G + 2 * fs + (int64_t)r0 * nh,
                       I->G + 2 * fs + (int64_t)(r0 + 1) * nh, t);
    }
  }
  const double bs0 = block_sum(s0, red);
  const double bs1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    I->part[2 * blockIdx.x] = bs0;
    I->part[2 * blockIdx.x + 1] = bs1;
  }
}

// Step setup, column part: g^ (stored for the whole step); FCH also the
// Laplacians of x0 (and of u^n for the midpoint rule) as spectral rows.
template <class PY, int MODEL>
__global__ __launch_bounds__(256) void k_col_setup(const InstDev* __restrict__ I) {
  extern __shared__ c2 smem[];
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int cb = blockDim.x / T;
  const int c = threadIdx.x % cb, t = threadIdx.x / cb;
  const int nh = I->nh;
  const int kx = blockIdx.x * cb + c;
  const bool valid = kx < nh;
  const int kxc = valid ? kx : nh - 1;
  c2* lds = smem + c * lds_len(N);
  const int64_t fs = I->field_stride;
  c2 v[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = I->G[(int64_t)(t + m * T) * nh + kxc];
  fft<PY, false>(v, lds, I->tw_y, t);
  if (valid) {
#pragma unroll
    for (int m = 0; m < RM; ++m) I->ghat[(int64_t)(t + m * T) * nh + kx] = v[m];
  }
  if constexpr (MODEL == MODEL_FCH) {
    const int nlap = I->theta != 1.0 ? 2 : 1;
    for (int f = 1; f <= nlap; ++f) {
#pragma unroll
      for (int m = 0; m < RM; ++m) v[m] = I->G[f * fs + (int64_t)(t + m * T) * nh + kxc];
      fft<PY, false>(v, lds, I->tw_y, t);
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const double k2 = wavenum2(I, kxc, t + m * T, N);
        v[m] = cscale(v[m], -k2 * I->inv_p);
      }
      fft<PY, true>(v, lds, I->tw_y, t);
      if (valid) {
#pragma unroll
        for (int m = 0; m < RM; ++m) I->G[f * fs + (int64_t)(t + m * T) * nh + kx] = v[m];
      }
    }
  }
}

// FCH step setup, second row part: Laplacians of x0 (and u^n) in real
// space, then the forward transforms that start iteration 0 (y_0 = x_0).
template <class PX>
__global__ __launch_bounds__(256) void k_row_start_fch(const InstDev* __restrict__ I) {
  extern __shared__ c2 smem[];
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (blockIdx.x * teams + team);
  const int nh = I->nh;
  const int64_t fs = I->field_stride;
  const double th = I->theta;
  const bool mp = th != 1.0;
  double lx[2][RM], lu[2][RM];
  if (!mp) {
    c2 v[RM];
    load_pack<PX>(v, I->G + fs + (int64_t)r0 * nh, I->G + fs + (int64_t)(r0 + 1) * nh, t);
    fft<PX, true>(v, lds, I->tw_x, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      lx[0][m] = v[m].x;
      lx[1][m] = v[m].y;
      lu[0][m] = 0.0;
      lu[1][m] = 0.0;
    }
  } else {
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      c2 v[RM];
      const int r = r0 + row;
      load_pack<PX>(v, I->G + fs + (int64_t)r * nh, I->G + 2 * fs + (int64_t)r * nh, t);
      fft<PX, true>(v, lds, I->tw_x, t);
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        lx[row][m] = v[m].x;
        lu[row][m] = v[m].y;
      }
    }
  }
  double vbs[2][RM];
#pragma unroll
  for (int row = 0; row < 2; ++row) {
    double lv[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int64_t idx = (int64_t)(r0 + row) * N + t + m * T;
      I->DX[0][idx] = lx[row][m];
      I->DX[2][idx] = lx[row][m];
      if (mp) I->dun[idx] = lu[row][m];
      const double x0 = I->X[0][idx];
      vbs[row][m] = mp ? th * x0 + (1.0 - th) * I->un[idx] : x0;
      lv[m] = mp ? th * lx[row][m] + (1.0 - th) * lu[row][m] : lx[row][m];
    }
    fch_forward_row<PX>(I, vbs[row], lv, lds, r0 + row, t);
  }
  pair_forward<PX>(I, vbs[0], vbs[1], lds, I->S + 2 * fs + (int64_t)r0 * nh,
                   I->S + 2 * fs + (int64_t)(r0 + 1) * nh, t);
}

}  // namespace pfch
