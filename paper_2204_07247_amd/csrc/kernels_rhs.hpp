// Right-hand side R(v) = M Delta mu(v) of the PDE on 2D grids and 3D PFC
// grids, and the error estimate of the adaptive step control (Sec. 3.1.2):
// the AM3 value needs R at the tentative and the two previous solutions.
//
// The transforms run in the instance's spectral workspace S (free between
// solves), with the tiled layout, column-0 packing and row pairing of the
// iteration kernels:
//   PFC: rows  S0 <- (v^3)^x, S1 <- v^x
//        cols  S0 <- R^ = -M q (N^ + (1 - eps - 2q + q^2) v^), inverse in y
//        rows  R  <- inverse x of S0
//   FCH: rows  S2 <- v^x
//        cols  S0 <- (Delta v)^, inverse in y
//        rows  Delta v <- inverse x of S0, then S0 <- F'^x, S1 <- p^x,
//              S2 <- v^x (p = -F'' omega - eta2 F', omega = eps^2 Delta v - F')
//        cols  S0 <- R^ = -M q (eps^2 q F'^ + p^ + (eps^4 q^2 - eps^2 eta1 q) v^)
//        rows  R  <- inverse x of S0
//   PFC 3D: rows  S0 <- (v^3)^x, S1 <- v^x (rows = Ny Nz, as above)
//           y     S0, S1 <- forward y-transforms (column 0 split)
//           z     S0 <- R^ = -M q (N^ + (1 - eps - 2q + q^2) v^), inverse in z
//           y     S0 <- inverse y-transform (column 0 merged)
//           rows  R  <- inverse x of S0
// The 1/(Nx Ny Nz) of the inverse transform is applied in k-space.  Every
// kernel takes a per-instance source (or destination) pointer; a null one
// skips the instance.  `spec`, when not null, replaces S (three fields of
// the instance's tiled spectral size) for every instance of the launch.
#pragma once
#include "kernels2d.hpp"
#include "kernels3d.hpp"

namespace pfch {

// The instance record staged in LDS, with the spectral workspace replaced by
// `spec` when that is not null (the allocation-free entry point passes its
// static scratch there).  Every thread of the block calls it.
__device__ __forceinline__ const InstDev* rhs_record(const InstDev* g, InstDev* rec, c2* spec) {
  stage_record(g, rec);
  if (spec) {
    if (threadIdx.x == 0) rec->S = spec;
    __syncthreads();
  }
  return rec;
}

template <class PX, int MODEL>
__global__ __launch_bounds__(256) void k_rhs_row_fwd(InstDev* const* __restrict__ grp,
                                                     const double* const* __restrict__ src, int bpi,
                                                     c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!src[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (lb * teams + team);
  const GLB double* v = gp(src[gi]);
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);
  double vb[2][RM];
#pragma unroll
  for (int row = 0; row < 2; ++row) {
#pragma unroll
    for (int m = 0; m < RM; ++m) vb[row][m] = v[(uint32_t)(r0 + row) * N + t + m * T];
  }
  if constexpr (MODEL == MODEL_PFC) {
    pfc_forward_pair<PX>(I, vb, tw, lds, r0, t);
  } else {
    GLB c2* S2 = gp(I->S) + 2 * I->field_stride;
    pair_forward<PX>(vb[0], vb[1], tw, lds, S2, r0, I->rows, t);
  }
}

// FCH middle row pass: Delta v from S0, then the pointwise terms at v and
// their forward x-transforms into S0, S1, S2.
template <class PX>
__global__ __launch_bounds__(256) void k_rhs_row_mid(InstDev* const* __restrict__ grp,
                                                     const double* const* __restrict__ src, int bpi,
                                                     c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!src[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (lb * teams + team);
  const GLB double* v = gp(src[gi]);
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);
  c2 z[RM];
  load_pack<PX>(z, gp(I->S), r0, I->rows, t);
  fft<PX, true>(z, lds, tw, t);
  double vb[2][RM], lv[2][RM];
#pragma unroll
  for (int row = 0; row < 2; ++row) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      vb[row][m] = v[(uint32_t)(r0 + row) * N + t + m * T];
      lv[row][m] = row ? z[m].y : z[m].x;
    }
  }
  fch_forward_pair<PX>(I, vb, lv, tw, lds, r0, t);
}

// Last row pass: R <- inverse x-transform of S0.
template <class PX>
__global__ __launch_bounds__(256) void k_rhs_row_inv(InstDev* const* __restrict__ grp,
                                                     double* const* __restrict__ dst, int bpi,
                                                     c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!dst[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (lb * teams + team);
  GLB double* out = gp(dst[gi]);
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);
  c2 z[RM];
  load_pack<PX>(z, gp(I->S), r0, I->rows, t);
  fft<PX, true>(z, lds, tw, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    out[(uint32_t)r0 * N + t + m * T] = z[m].x;
    out[(uint32_t)(r0 + 1) * N + t + m * T] = z[m].y;
  }
}

// Column pass: y-transforms of the input fields, a real symbol per field
// and logical column, summed, inverse y-transform into S0.
//   STAGE 0 (PFC): fields S0 = N^, S1 = v^.
//   STAGE 1 (FCH): field S2 = v^, symbol of Delta.
//   STAGE 2 (FCH): fields S0 = F'^, S1 = p^, S2 = v^.
template <class PY, int MODEL, int STAGE>
__global__ __launch_bounds__(512) void k_rhs_col(InstDev* const* __restrict__ grp,
                                                 const double* const* __restrict__ src, int bpi,
                                                 c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!src[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  constexpr int F0 = STAGE == 1 ? 2 : 0;
  constexpr int F1 = MODEL == MODEL_PFC ? 2 : 3;  // fields F0 .. F1-1
  const int rows = N;
  const ColPos pos = col_pos(T, I->nh / TW, lb);
  const int t = pos.t, kp = pos.kp;
  c2* lds = smem + pos.c * lds_len(N);
  const bool special = kp == 0;
  const bool blk0 = lb == 0;
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* S = gp(I->S);
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);
  const double kxn2 = (0.5 * I->nx * I->kx_scale) * (0.5 * I->nx * I->kx_scale);
  const double kx2 = (kp * I->kx_scale) * (kp * I->kx_scale);
  const double e2 = I->eps * I->eps, mp = -I->mobility * I->inv_p;
  auto q_of = [&](int ky) {
    const double a = (ky <= N / 2 ? ky : ky - N) * I->ky_scale;
    return kx2 + a * a;
  };
  auto q_col0 = [&](int ky) {
    const double a = (ky <= N / 2 ? ky : ky - N) * I->ky_scale;
    return a * a;
  };
  auto coef = [&](int f, double q) -> double {
    if constexpr (MODEL == MODEL_PFC) {
      return f == 0 ? mp * q : mp * q * (1.0 - I->eps - 2.0 * q + q * q);
    } else if constexpr (STAGE == 1) {
      return -I->inv_p * q;
    } else {
      if (f == 0) return mp * e2 * q * q;
      if (f == 1) return mp * q;
      return mp * q * (e2 * e2 * q * q - e2 * I->eta1 * q);
    }
  };
  c2 v[RM], acc[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) acc[m] = c2{0.0, 0.0};
#pragma unroll
  for (int f = F0; f < F1; ++f) {
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = gload(S + f * fs + sidx(rows, t + m * T, kp));
    fft<PY, false>(v, lds, tw, t);
    const int tf = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const double q = q_of(tf + m * T);
      const double c = special ? 0.5 * (coef(f, q) + coef(f, q + kxn2)) : coef(f, q);
      acc[m] = cadd(acc[m], cscale(v[m], c));
    }
    if (blk0)
      col0_mirror<PY>(v, smem, special, t, [&](int m, c2 w) {
        const double q = q_col0(opaque(t + m * T));
        acc[m] = cadd(acc[m], cscale(w, 0.5 * (coef(f, q) - coef(f, q + kxn2))));
      });
  }
  fft<PY, true>(acc, lds, tw, t);
  const int ts = opaque(t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(S + sidx(rows, ts + m * T, kp), acc[m]);
}

// 3D y-pass of R(v): forward y-transforms of S0 and S1 with column 0 split,
// or (INV) column 0 merged and the inverse y-transform of S0; the geometry
// of k_y3_iter.
template <class PY, bool INV>
__global__ __launch_bounds__(512) void k_rhs_y3(InstDev* const* __restrict__ grp,
                                                const double* const* __restrict__ src, int bpi, c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!src[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int rows = I->rows;
  const Y3Pos pos = y3_pos(T, I->nh / TW, lb);
  const int t = pos.t, kp = pos.kp, r0 = pos.z * N;
  c2* lds = smem + pos.c * lds_len(N);
  const bool col0 = kp == 0;
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* S = gp(I->S);
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);
  constexpr int NF = INV ? 1 : 2;
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    GLB c2* F = S + f * fs;
    c2 v[RM];
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = gload(F + sidx(rows, r0 + t + m * T, kp));
    if (INV && pos.has_col0) col0_merge<PY>(v, smem, col0, t);
    fft<PY, INV>(v, lds, tw, t);
    if (!INV && pos.has_col0) col0_split<PY>(v, smem, col0, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) gstore(F + sidx(rows, r0 + t + m * T, kp), v[m]);
  }
}

// 3D z-pass of R(v): forward z-transforms of N^ (S0) and v^ (S1), the
// symbol of R per logical column (packed slots through the mirror kz -> -kz,
// as in k_z3_iter), inverse z-transform into S0.
template <class PZ>
__global__ __launch_bounds__(512) void k_rhs_z3(InstDev* const* __restrict__ grp,
                                                const double* const* __restrict__ src, int bpi, c2* spec) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  if (!src[gi]) return;
  const InstDev* __restrict__ I = rhs_record(grp[gi], &rec, spec);
  constexpr int N = PZ::N, T = PZ::T, RM = PZ::RMAX;
  const int rows = I->rows, ny = I->ny;
  const Z3Pos pos = z3_pos(T, I->nh / TW, ny, lb);
  const int t = pos.t, kp = pos.kp, ky = pos.ky;
  c2* lds = smem + pos.c * lds_len(N);
  const bool pair = kp == 0 && (ky == 0 || 2 * ky == ny);
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* S = gp(I->S);
  Twiddles<PZ> tw;
  load_twiddles<PZ>(tw, I->tw_z, t);
  const double mp = -I->mobility * I->inv_p, e1 = 1.0 - I->eps;
  const double kxn2 = (0.5 * I->nx * I->kx_scale) * (0.5 * I->nx * I->kx_scale);
  auto at = [&](int tt, int m) { return sidx(rows, ky + (tt + m * T) * ny, kp); };
  auto coef = [&](int f, double q) -> double { return f == 0 ? mp * q : mp * q * (e1 - 2.0 * q + q * q); };
  c2 v[RM], acc[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) acc[m] = c2{0.0, 0.0};
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = gload(S + f * fs + at(tl, m));
    fft<PZ, false>(v, lds, tw, t);
    const int tf = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const double q = q3(I, kp, ky, tf + m * T);
      const double c = pair ? 0.5 * (coef(f, q) + coef(f, q + kxn2)) : coef(f, q);
      acc[m] = cadd(acc[m], cscale(v[m], c));
    }
    if (pos.has_pair)
      col0_mirror<PZ>(v, lds, pair, t, [&](int m, c2 w) {
        const double q = q3(I, 0, ky, opaque(t + m * T));
        acc[m] = cadd(acc[m], cscale(w, 0.5 * (coef(f, q) - coef(f, q + kxn2))));
      });
  }
  fft<PZ, true>(acc, lds, tw, t);
  const int ts = opaque(t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(S + at(ts, m), acc[m]);
}

// Error estimate of one attempt: u^ = sum_k w[k] f[k] over up to six fields
// (u^n, u^{n-1}, u^{n-2}, R~, R(u^n), R(u^{n-1}); a null pointer or zero
// weight drops a term), then per block the partial sums of (u~ - u^)^2 and
// u^2 in a fixed order.  Grid (EST_BLOCKS, instances).
constexpr int EST_BLOCKS = 128, EST_THREADS = 256;
struct EstArgs {
  const double* ut;  // tentative solution; null = skip the instance
  const double* f[6];
  double w[6];
  int64_t n;
};

__global__ __launch_bounds__(EST_THREADS) void k_adapt_est(const EstArgs* __restrict__ args,
                                                           double* __restrict__ part) {
  __shared__ double red[EST_THREADS / 64];
  const EstArgs& A = args[blockIdx.y];
  if (!A.ut) return;
  const GLB double* ut = gp(A.ut);
  const int64_t n = A.n;
  double se = 0.0, sh = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    double h = 0.0;
#pragma unroll
    for (int j = 0; j < 6; ++j)
      if (A.f[j] && A.w[j] != 0.0) h += A.w[j] * gp(A.f[j])[k];
    const double e = ut[k] - h;
    se += e * e;
    sh += h * h;
  }
  const double be = block_sum(se, red);
  const double bh = block_sum(sh, red);
  if (threadIdx.x == 0) {
    double* p = part + (int64_t)blockIdx.y * 2 * gridDim.x;
    p[blockIdx.x] = be;
    p[gridDim.x + blockIdx.x] = bh;
  }
}

}  // namespace pfch
