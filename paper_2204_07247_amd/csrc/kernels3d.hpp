// Three-dimensional PFC: the y- and z-passes of a PAGD iteration.
//
// Real fields are [Nz][Ny][Nx] (x fastest); the x-pass (row kernel) is the
// two-dimensional one with rows = Ny * Nz, row index r = z * Ny + y.  Spectral
// fields keep the tiled layout of the 2D path with that row index.  One
// iteration is four kernels:
//   k_y3_iter<fwd>  forward y-transform of the row-transformed fields,
//   k_z3_iter       forward z-transform, k-space residual and
//                   preconditioner (as in the 2D column kernel, with
//                   |k|^2 = kx^2 + ky^2 + kz^2), inverse z-transform of d^,
//   k_y3_iter<inv>  inverse y-transform of d^,
//   k_row_iter      inverse x-transform, update, nonlinear terms, forward
//                   x-transform (shared with 2D).
//
// Physical column 0 holds the kx = 0 and kx = Nx/2 columns packed as
// C0 + i CN (both real in y and z).  Between the y-passes it is kept split:
// for 0 < ky < Ny/2, slot ky holds the y-transform C0^(ky) and slot Ny - ky
// holds CN^(ky) (their values at -ky are the conjugates); slots 0 and Ny/2
// keep the packed pair, which is real in y but not in z, and the z kernel
// separates it through the mirror kz -> -kz as the 2D column kernel does.
#pragma once
#include "kernels2d.hpp"

namespace pfch {

// y-pass geometry: `cb` physical columns of one 4-wide tile at one z per
// block; blocks ordered (z, tile, part of tile).
struct Y3Pos {
  int c, t, kp, z;
  bool has_col0;  // the block holds physical column 0 (block-uniform)
};
__device__ __forceinline__ Y3Pos y3_pos(int T, int ntiles, int lb) {
  const int cb = blockDim.x / T;
  Y3Pos p;
  p.c = threadIdx.x % cb;
  p.t = threadIdx.x / cb;
  const int per_tile = TW / cb;
  const int per_z = ntiles * per_tile;
  p.z = lb / per_z;
  const int r = lb - p.z * per_z;
  const int kp0 = (r / per_tile) * TW + (r % per_tile) * cb;
  p.kp = kp0 + p.c;
  p.has_col0 = kp0 == 0;
  return p;
}

// Split / merge of physical column 0 around the z-passes (see the file
// comment).  v holds the column's y-transform at ky = t + m T.  Every thread
// of the block calls these (they contain barriers); only `mine` changes v.
template <class P>
__device__ __forceinline__ void col0_split(c2 (&v)[P::RMAX], c2* lds0, bool mine, int t) {
  constexpr int N = P::N, T = P::T;
  if (mine) {
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) lds0[lds_idx(t + m * T)] = v[m];
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) {
      const int k = t + m * T;
      if (k == 0 || 2 * k == N) continue;
      const c2 a = v[m], w = lds0[lds_idx(N - k)];  // P^(k), P^(N-k)
      if (2 * k < N) {
        v[m] = c2{0.5 * (a.x + w.x), 0.5 * (a.y - w.y)};  // (P(k) + conj P(-k)) / 2
      } else {
        // slot k holds CN^(N-k) = -i (P(N-k) - conj P(k)) / 2
        const c2 d = c2{w.x - a.x, w.y + a.y};
        v[m] = c2{0.5 * d.y, -0.5 * d.x};
      }
    }
  }
  __syncthreads();
}

template <class P>
__device__ __forceinline__ void col0_merge(c2 (&v)[P::RMAX], c2* lds0, bool mine, int t) {
  constexpr int N = P::N, T = P::T;
  if (mine) {
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) lds0[lds_idx(t + m * T)] = v[m];
  }
  __syncthreads();
  if (mine) {
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) {
      const int k = t + m * T;
      if (k == 0 || 2 * k == N) continue;
      const c2 a = v[m], w = lds0[lds_idx(N - k)];
      if (2 * k < N)
        v[m] = c2{a.x - w.y, a.y + w.x};  // C0(k) + i CN(k)
      else
        v[m] = c2{w.x + a.y, a.x - w.y};  // conj C0(N-k) + i conj CN(N-k)
    }
  }
  __syncthreads();
}

// y-pass of one iteration.  Forward: both PFC fields (N^ and v_breve^ after
// the x-transform), then column 0 split.  Inverse: column 0 merged, then the
// inverse y-transform of d^ (field 0).  In place.
template <class PY, bool INV>
__global__ __launch_bounds__(512) void k_y3_iter(const InstDev* const* __restrict__ grp, int bpi, int l,
                                                 int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int rows = I->rows;
  const Y3Pos pos = y3_pos(T, I->nh / TW, gpos.lb);
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

// Step setup, y part: forward y-transform of the x-transformed step
// constant g into g^ (column 0 split).  Block 0 sums the averaged-Newton
// partial sums of the row setup.
template <class PY>
__global__ __launch_bounds__(512) void k_y3_setup(InstDev* const* __restrict__ grp, int bpi) {
  extern __shared__ c2 smem[];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  InstDev* __restrict__ I = grp[gi];
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int rows = I->rows;
  const Y3Pos pos = y3_pos(T, I->nh / TW, lb);
  const int t = pos.t, kp = pos.kp, r0 = pos.z * N;
  c2* lds = smem + pos.c * lds_len(N);
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);
  if (lb == 0) finish_betas(I);
  c2 v[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = gload(gp(I->G) + sidx(rows, r0 + t + m * T, kp));
  fft<PY, false>(v, lds, tw, t);
  if (pos.has_col0) col0_split<PY>(v, smem, kp == 0, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(gp(I->ghat) + sidx(rows, r0 + t + m * T, kp), v[m]);
}

// z-pass geometry: the 4 physical columns of a tile times `kyb` consecutive
// ky per block (4 kyb columns of T threads; a z-slice of the block's columns
// is 64 kyb contiguous bytes).  Blocks ordered (ky block, tile).
struct Z3Pos {
  int c, t, kp, ky;
  bool has_pair;  // the block holds a packed pair column (block-uniform)
};
__device__ __forceinline__ Z3Pos z3_pos(int T, int ntiles, int ny, int lb) {
  const int ncol = blockDim.x / T, kyb = ncol / TW;
  Z3Pos p;
  p.c = threadIdx.x % ncol;
  p.t = threadIdx.x / ncol;
  const int tile = lb % ntiles, kyblk = lb / ntiles;
  p.kp = tile * TW + (p.c % TW);
  p.ky = kyblk * kyb + p.c / TW;
  const int ky0 = kyblk * kyb, kyh = ny / 2;
  p.has_pair = tile == 0 && (ky0 == 0 || (kyh >= ky0 && kyh < ky0 + kyb));
  return p;
}

// |k|^2 of the logical column behind physical slot (kp, ky) at kz.  For
// kp = 0: slots 0 < ky < Ny/2 are kx = 0, slots ky > Ny/2 are kx = Nx/2 at
// y-wavenumber Ny - ky (same |ky|), and the packed slots 0 and Ny/2 report
// kx = 0 (the kx = Nx/2 part is added through the mirror).
__device__ __forceinline__ double q3(const InstDev* I, int kp, int ky, int kz) {
  const int ny = I->ny, nz = I->nz;
  double kx2;
  if (kp > 0) {
    const double a = kp * I->kx_scale;
    kx2 = a * a;
  } else if (2 * ky > ny) {
    const double a = 0.5 * I->nx * I->kx_scale;
    kx2 = a * a;
  } else {
    kx2 = 0.0;
  }
  const double b = (ky <= ny / 2 ? ky : ky - ny) * I->ky_scale;
  const double c = (kz <= nz / 2 ? kz : kz - nz) * I->kz_scale;
  return kx2 + b * b + c * c;
}

// z-pass of one PFC iteration: forward z-transforms of N^ and v_breve^, then
//   d^ = -(1/(P Lq)) [ (a/theta v^ + g^)/M + q N^ + q (1 - eps - 2q + q^2) v^ ],
// zero at k = 0, and the inverse z-transform of d^ into field 0.
template <class PZ>
__global__ __launch_bounds__(512) void k_z3_iter(const InstDev* const* __restrict__ grp, int bpi, int l,
                                                 int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PZ::N, T = PZ::T, RM = PZ::RMAX;
  const int rows = I->rows, ny = I->ny;
  const Z3Pos pos = z3_pos(T, I->nh / TW, ny, gpos.lb);
  const int t = pos.t, kp = pos.kp, ky = pos.ky;
  c2* lds = smem + pos.c * lds_len(N);
  const bool pair = kp == 0 && (ky == 0 || 2 * ky == ny);
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* S = gp(I->S);
  Twiddles<PZ> tw;
  load_twiddles<PZ>(tw, I->tw_z, t);
  double bm2, b0, b2, b4;
  betas(I, bm2, b0, b2, b4);
  // the record's scalars in scalar registers
  bm2 = uni_d(bm2);
  b0 = uni_d(b0);
  b2 = uni_d(b2);
  b4 = uni_d(b4);
  const double thl = uni_d(I->theta_l), inv_m = uni_d(I->inv_mobility), aot = uni_d(I->a_over_theta);
  const double inv_p = uni_d(I->inv_p), e1 = 1.0 - uni_d(I->eps);
  const double hx = 0.5 * uni_i(I->nx) * uni_d(I->kx_scale);
  const double kxn2 = hx * hx;
  // |k|^2 at kx = 0 of a pair slot (ky = 0 or ny/2) at kz
  const double kyp = ky * uni_d(I->ky_scale), kzs = uni_d(I->kz_scale);
  const int nzu = uni_i(I->nz);
  auto q_pair = [&](int kz) {
    const double c = (kz <= nzu / 2 ? kz : kz - nzu) * kzs;
    return kyp * kyp + c * c;
  };
  // Element m of this thread: z index tt + m T for a thread index tt.  Each
  // phase takes its own opaque copy of t so that addresses and wavenumbers
  // are recomputed there instead of being held live across the transforms.
  auto at = [&](int tt, int m) { return sidx(rows, ky + (tt + m * T) * ny, kp); };
  auto coef = [&](int f, double q) -> double {
    return f == 1 ? inv_m * aot + q * (e1 - 2.0 * q + q * q) : q;
  };
  // scale by -1/(P Lq), zero at k = 0
  int bad = 0;
  auto scale = [&](double q) -> double {
    const double Lq = bm2 + thl * q * (b0 + b2 * q + b4 * q * q);
    const bool pos = q > 0.0;
    bad |= pos & !(Lq > 0.0);
    const double r = -inv_p * rcp_pos(Lq);
    return pos ? r : 0.0;
  };
  // The pair slots take symbol times scale per logical column (kx = 0 and
  // kx = nx/2, whose symbols differ by orders of magnitude) inside the
  // mirror exchanges and are not scaled again; `keep` is 0 there.
  auto sig = [&](int f, double q) { return coef(f, q) * scale(q); };
  const double keep = pair ? 0.0 : 1.0;

  // With up to 8 elements per thread the next field is loaded before the
  // transform of the current one; with more, after it (registers).
  constexpr bool PREFETCH = RM <= 8;
  c2 v[RM], nxt[PREFETCH ? RM : 1], acc[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    v[m] = gload(S + at(t, m));
    acc[m] = c2{0.0, 0.0};
  }
#pragma unroll
  for (int f = 0; f < 2; ++f) {
    if constexpr (PREFETCH) {
#pragma unroll
      for (int m = 0; m < RM; ++m) nxt[m] = f == 0 ? gload(S + fs + at(t, m)) : gload(gp(I->ghat) + at(t, m));
    }
    fft<PZ, false>(v, lds, tw, t);
    const int tf = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = cadd(acc[m], cscale(v[m], keep * coef(f, q3(I, kp, ky, tf + m * T))));
    if (pos.has_pair)
      col0_pair<PZ>(v, lds, pair, t, [&](int m, c2 own, c2 w) {
        const double q = q_pair(opaque(t + m * T));
        const double s0 = sig(f, q), sn = sig(f, q + kxn2);
        acc[m] = cadd(acc[m], cadd(cscale(own, 0.5 * (s0 + sn)), cscale(w, 0.5 * (s0 - sn))));
      });
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      if constexpr (PREFETCH)
        v[m] = nxt[m];
      else
        v[m] = f == 0 ? gload(S + fs + at(tf, m)) : gload(gp(I->ghat) + at(tf, m));
    }
  }
#pragma unroll
  for (int m = 0; m < RM; ++m) acc[m] = cadd(acc[m], cscale(v[m], keep * inv_m));
  if (pos.has_pair)
    col0_pair<PZ>(v, lds, pair, t, [&](int m, c2 own, c2 w) {
      const double q = q_pair(opaque(t + m * T));
      const double s0 = inv_m * scale(q), sn = inv_m * scale(q + kxn2);
      acc[m] = cadd(acc[m], cadd(cscale(own, 0.5 * (s0 + sn)), cscale(w, 0.5 * (s0 - sn))));
    });
  const int te = opaque(t);
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = pair ? acc[m] : cscale(acc[m], scale(q3(I, kp, ky, te + m * T)));
  fft<PZ, true>(v, lds, tw, t);
  const int ts = opaque(t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(S + at(ts, m), v[m]);
  if (bad) atomicOr(I->flags, FLAG_PRECOND);
}

// Step setup, z part: forward z-transform of g^ in place.
template <class PZ>
__global__ __launch_bounds__(512) void k_z3_setup(InstDev* const* __restrict__ grp, int bpi) {
  extern __shared__ c2 smem[];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  const InstDev* __restrict__ I = grp[gi];
  constexpr int N = PZ::N, T = PZ::T, RM = PZ::RMAX;
  const int rows = I->rows, ny = I->ny;
  const Z3Pos pos = z3_pos(T, I->nh / TW, ny, lb);
  const int t = pos.t, kp = pos.kp, ky = pos.ky;
  c2* lds = smem + pos.c * lds_len(N);
  GLB c2* G = gp(I->ghat);
  Twiddles<PZ> tw;
  load_twiddles<PZ>(tw, I->tw_z, t);
  c2 v[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = gload(G + sidx(rows, ky + (t + m * T) * ny, kp));
  fft<PZ, false>(v, lds, tw, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(G + sidx(rows, ky + (t + m * T) * ny, kp), v[m]);
}

}  // namespace pfch
