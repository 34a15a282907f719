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
// Layouts.  Real fields are [rows][nx] (x fastest).  A row's half spectrum
// has nx/2 + 1 entries of which the first (kx = 0) and the last (kx = nx/2)
// are real for real data; they share physical column 0 as (A[0], A[nx/2]),
// so a spectral row has exactly H = nx/2 complex entries.  Spectral fields
// are stored in column tiles of TW = 4 columns: element (row, kp) lives at
// ((kp / 4) * rows + row) * 4 + kp % 4.  A column tile is one contiguous
// block (what the column kernel streams), and a row pair writes whole
// 128-byte lines into every tile.
#pragma once
#include "fft.hpp"
#include "pfch_dev.hpp"

namespace pfch {

constexpr int TW = 4;

__device__ __forceinline__ uint64_t dbits(double v) { return (uint64_t)__double_as_longlong(v); }

// Element offset of (row, kp) in a spectral field: tiles of TW = 4 physical
// columns, each tile's rows in order, and in a 128-byte line the row pair
// (2i, 2i + 1) of the tile's four columns, column-major (the two rows of one
// column adjacent).  A column pass then reads and writes 32 contiguous bytes
// per line and column, a row-pair pass whole lines.  32-bit: a field holds
// at most rows * H <= 2^31 / 16 elements, which keeps the base pointer in
// scalar registers and one offset register per access.
__device__ __forceinline__ uint32_t sidx(int rows, int row, int kp) {
  return ((uint32_t)(kp >> 2) * (uint32_t)rows + (uint32_t)(row & ~1)) * TW + (uint32_t)(kp & 3) * 2 +
         (uint32_t)(row & 1);
}

// The value of lane ^ 1 (both lanes active).
__device__ __forceinline__ double lane_pair_swap(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, 0xB1, 0xF, 0xF, false);  // quad_perm(1,0,3,2)
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// An opaque copy of v: keeps the compiler from hoisting work that depends
// on it out of a rarely taken branch (and holding the results live across
// barriers).
__device__ __forceinline__ int opaque(int v) { return opaque_i(v); }

// Block-uniform copies (the value of the first active lane) of values every
// lane of the block has read alike: held in scalar registers rather than one
// vector register per lane.  Applied to values already loaded (from the LDS
// copy of the instance record), so that no record field is ever read
// through the scalar cache, which does not see what earlier kernels of the
// same graph wrote.
__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ uint64_t uni_u64(uint64_t b) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ double uni_d(double v) { return __longlong_as_double((long long)uni_u64(dbits(v))); }
template <class T>
__device__ __forceinline__ T* uni_p(T* p) {
  return (T*)(uintptr_t)uni_u64((uint64_t)(uintptr_t)p);
}

// Grouped launches: one launch covers every instance of a group (same model
// and grid); block b works on instance b / bpi as its local block b % bpi.
struct GroupPos {
  const InstDev* I;
  int lb;  // block index within the instance
};
__device__ __forceinline__ GroupPos group_pos(const InstDev* const* __restrict__ grp, int bpi) {
  const int gi = blockIdx.x / bpi;
  return GroupPos{grp[gi], (int)blockIdx.x - gi * bpi};
}

// The instance record copied into LDS at kernel entry: all of its fields in
// one round trip of vector loads (which see what earlier kernels of the
// same graph wrote), after which every field read is an LDS read rather
// than a dependent global load.  Every thread of the block calls it; the
// record is read-only here (writes go to the global record).
__device__ __forceinline__ const InstDev* stage_record(const InstDev* g, InstDev* rec) {
  static_assert(sizeof(InstDev) % 8 == 0, "the record is staged in 8-byte words");
  constexpr int W = (int)(sizeof(InstDev) / 8);
  const GLB uint64_t* src = gp(reinterpret_cast<const uint64_t*>(g));
  uint64_t* dst = reinterpret_cast<uint64_t*>(rec);
  // unconditional (threads past the record repeat its last word), so that
  // the record's load is not held behind a branch on the block size
  const int w0 = min((int)threadIdx.x, W - 1);
  dst[w0] = src[w0];
  for (int w = threadIdx.x + blockDim.x; w < W; w += blockDim.x) dst[w] = src[w];
  __syncthreads();
  return rec;
}

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

// ---------------------------------------------------------------------------
// Row-side packing.
// ---------------------------------------------------------------------------
// Z[k] = A[k] + i B[k] over the full length from the Hermitian half spectra
// of rows r0 (A) and r0 + 1 (B) of F, r0 even.  With teams of whole waves
// the lanes of a pair (k, k + 1, k even) load the columns of both their
// elements as two 32-byte pieces (each lane one row of each) and exchange
// the halves they hold for each other; smaller teams (short rows, several
// row pairs per wave) load A[k] and B[k] directly, which measured faster
// there.
template <class P>
__device__ __forceinline__ void load_pack(c2 (&v)[P::RMAX], const GLB c2* __restrict__ F, int r0, int rows,
                                          int t) {
  constexpr int N = P::N, T = P::T;
  auto col = [](int k) { return k == N / 2 ? 0 : (k > N / 2 ? N - k : k); };
#pragma unroll
  for (int m = 0; m < P::RMAX; ++m) {
    const int k = t + m * T;
    c2 a, b;
    if constexpr (T % 2 == 0 && T >= 64) {
      const bool odd = k & 1;
      const int ke = k & ~1;
      const int row = r0 + (odd ? 1 : 0);
      const c2 v1 = gload(F + sidx(rows, row, col(ke)));
      const c2 v2 = gload(F + sidx(rows, row, col(ke + 1)));
      const c2 send = odd ? v1 : v2;
      const c2 recv = c2{lane_pair_swap(send.x), lane_pair_swap(send.y)};
      a = odd ? recv : v1;
      b = odd ? v2 : recv;
    } else {
      a = gload(F + sidx(rows, r0, col(k)));
      b = gload(F + sidx(rows, r0 + 1, col(k)));
    }
    if (k == 0 || k == N / 2) {  // column 0 holds (A[0], A[N/2]) and (B[0], B[N/2])
      a = c2{k == 0 ? a.x : a.y, 0.0};
      b = c2{k == 0 ? b.x : b.y, 0.0};
    } else if (k > N / 2) {
      a.y = -a.y;
      b.y = -b.y;
    }
    v[m] = c2{a.x - b.y, a.y + b.x};
  }
}

// After the forward transform of Z = a + i b (a, b the real rows r0, r0 + 1,
// r0 even): store the half spectra A[k] = (Z[k] + conj Z[N-k]) / 2 into row
// r0 and B[k] = -i (Z[k] - conj Z[N-k]) / 2 into row r0 + 1 of F (k = 0 and
// N/2 packed in column 0).  With teams of whole waves, lane s of round m
// takes the s-th 16-byte slot of the row pair's lines (k = s / 2, row
// r0 + s % 2), so that each store instruction writes whole lines; the lanes
// of a pair read Z[k] and Z[N-k] from LDS and exchange them.  Smaller teams
// store A[k] and B[k] from one lane.
template <class P>
__device__ __forceinline__ void unpack_store(const c2 (&v)[P::RMAX], c2* lds, GLB c2* __restrict__ F, int r0,
                                             int rows, int t) {
  constexpr int N = P::N, T = P::T;
#pragma unroll
  for (int m = 0; m < P::RMAX; ++m) lds[lds_idx(t + m * T)] = v[m];
  __syncthreads();
  if constexpr (T % 2 == 0 && T >= 64) {
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) {
      const int sl = t + m * T, k = sl >> 1;
      const bool odd = sl & 1;
      const c2 mine = lds[lds_idx(odd ? (k == 0 ? N / 2 : N - k) : k)];
      const c2 other = c2{lane_pair_swap(mine.x), lane_pair_swap(mine.y)};
      const c2 z = odd ? other : mine, w = odd ? mine : other;
      c2 out;
      if (k == 0)
        out = odd ? c2{z.y, w.y} : c2{z.x, w.x};  // (Im / Re Z[0], Im / Re Z[N/2])
      else
        out = odd ? c2{0.5 * (z.y + w.y), -0.5 * (z.x - w.x)} : c2{0.5 * (z.x + w.x), 0.5 * (z.y - w.y)};
      gstore(F + sidx(rows, r0 + (odd ? 1 : 0), k), out);
    }
  } else {
#pragma unroll
    for (int m = 0; m < P::RMAX / 2; ++m) {
      const int k = t + m * T;
      const c2 z = lds[lds_idx(k)];
      const c2 w = lds[lds_idx(k == 0 ? N / 2 : N - k)];
      c2 A, B;
      if (k == 0) {
        A = c2{z.x, w.x};
        B = c2{z.y, w.y};
      } else {
        A = c2{0.5 * (z.x + w.x), 0.5 * (z.y - w.y)};
        B = c2{0.5 * (z.y + w.y), -0.5 * (z.x - w.x)};
      }
      gstore(F + sidx(rows, r0, k), A);
      gstore(F + sidx(rows, r0 + 1, k), B);
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Column-side helpers.
// ---------------------------------------------------------------------------
// |k|^2 for logical column kx and row index ky.
__device__ __forceinline__ double wavenum2(const InstDev* I, int kx, int ky, int ny) {
  const int kyp = ky <= ny / 2 ? ky : ky - ny;
  const double ax = kx * I->kx_scale, ay = kyp * I->ky_scale;
  return ax * ax + ay * ay;
}

// Averaged-Newton constants (beta_-2, beta_0, beta_2, beta_4).  beta_0 and
// beta_2 are the grid means of Sec. 3.4.1 at the step's initial guess,
// summed once per step in a fixed order by the setup column kernel.
__device__ __forceinline__ void betas(const InstDev* I, double& bm2, double& b0, double& b2,
                                      double& b4) {
  if (I->resid) {  // identity preconditioner (Lq = q): d^ = r^, the residual itself
    bm2 = 0.0;
    b0 = 1.0 / I->theta_l;
    b2 = 0.0;
    b4 = 0.0;
    return;
  }
  bm2 = I->a / I->mobility;
  b0 = I->beta0;
  if (I->model == MODEL_PFC) {
    b2 = -2.0;
    b4 = 1.0;
  } else {
    const double e2 = I->eps * I->eps;
    b2 = I->beta2;
    b4 = e2 * e2;
  }
}

// Called by every thread of one block.  The partial sums are added in index
// order by one thread (the order the host's report uses), staged through LDS
// in chunks so that the loads are issued by the whole block.
// The step's averaged-Newton constants from the set-up's partial sums
// (strided per thread, then the block's fixed reduction tree, so every block
// gets the same value), returned to every thread of the block (all must
// call it).
__device__ __forceinline__ void sum_betas(const InstDev* I, double& b0, double& b2) {
  if (I->imex) {
    b0 = I->imex_b0;
    b2 = I->imex_b2;
    return;
  }
  __shared__ double red[16];
  __shared__ double out[2];
  double s0 = 0.0, s1 = 0.0;
  const int np = I->nparts;
  for (int k = threadIdx.x; k < np; k += blockDim.x) {
    s0 += I->part[2 * k];
    s1 += I->part[2 * k + 1];
  }
  const double t0 = block_sum(s0, red);
  const double t1 = block_sum(s1, red + 8);
  if (threadIdx.x == 0) {
    out[0] = fabs(t0 * I->inv_p);
    out[1] = fabs(t1 * I->inv_p);
  }
  __syncthreads();
  b0 = out[0];
  b2 = out[1];
  __syncthreads();
}

__device__ __forceinline__ void finish_betas(InstDev* I) {
  double b0, b2;
  sum_betas(I, b0, b2);
  if (threadIdx.x == 0) {
    I->beta0 = b0;
    I->beta2 = b2;
  }
}

// First column iteration of a step whose column set-up was folded in: the
// constants come from the partial sums (block 0 also stores them for the
// later iterations in `home`, the instance's global record).  Uniform per
// block: every thread calls it.
__device__ __forceinline__ void fold_betas(const InstDev* I, InstDev* home, bool blk0, double& b0,
                                           double& b2) {
  double f0, f2;
  sum_betas(I, f0, f2);
  if (!I->resid) {
    b0 = f0;
    if (I->model == MODEL_FCH) b2 = f2;
  }
  if (blk0 && threadIdx.x == 0) {
    home->beta0 = f0;
    home->beta2 = f2;
  }
}

// Column block geometry: `cb` physical columns per block (1, 2 or 4 of a
// tile).  Blocks sharing a tile are placed on the same XCD (block ids go
// round-robin over the 8 XCDs) when the tile count allows it.
struct ColPos {
  int c, t, kp;
};
__device__ __forceinline__ ColPos col_pos(int T, int ntiles, int lb) {
  const int cb = blockDim.x / T;
  ColPos p;
  p.c = threadIdx.x % cb;
  p.t = threadIdx.x / cb;
  const int per_tile = TW / cb;
  int tile, sub;
  if (per_tile > 1 && (ntiles & 7) == 0) {
    const int g = lb / (8 * per_tile), r = lb % (8 * per_tile);
    tile = g * 8 + (r & 7);
    sub = r >> 3;
  } else {
    tile = lb / per_tile;
    sub = lb % per_tile;
  }
  p.kp = tile * TW + sub * cb + p.c;
  return p;
}

// Physical column 0 packs the logical columns kx = 0 and kx = N/2:
// P^(ky) = F0^(ky) + i FN^(ky), both transforms of real sequences.  A real
// symbol applied per logical column, c0(ky) to F0^ and cN(ky) to FN^, acts
// on the packed values as
//   c0 F0^ + i cN FN^ = (c0 + cN)/2 P^(ky) + (c0 - cN)/2 conj(P^(-ky)).
// col0_mirror hands conj(P^(-ky)) of column 0's own values to `use`.  Every
// thread of the block must call it; only column 0's team (`mine`) calls
// `use`.
template <class P, class F>
__device__ __forceinline__ void col0_mirror(const c2 (&v)[P::RMAX], c2* lds0, bool mine, int t, F use) {
  constexpr int N = P::N, T = P::T;
  // Indices from opaque copies of t: computed inside the (rare) branches
  // rather than ahead of them and held live across the transforms.
  if (mine) {
    const int ts = opaque_i(t);
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) lds0[lds_idx(ts + m * T)] = v[m];
  }
  __syncthreads();
  if (mine) {
    const int tl = opaque_i(t);
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) {
      const int ky = tl + m * T;
      const c2 w = lds0[lds_idx(ky == 0 ? 0 : N - ky)];
      use(m, c2{w.x, -w.y});
    }
  }
  __syncthreads();
}

// As col0_mirror, handing `use` the own value P^(ky) read back from LDS
// together with conj(P^(-ky)), so that the caller's registers of v are free
// across the exchange.
template <class P, class F>
__device__ __forceinline__ void col0_pair(const c2 (&v)[P::RMAX], c2* lds0, bool mine, int t, F use) {
  constexpr int N = P::N, T = P::T;
  if (mine) {
    const int ts = opaque_i(t);
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) lds0[lds_idx(ts + m * T)] = v[m];
  }
  __syncthreads();
  if (mine) {
    const int tl = opaque_i(t);
#pragma unroll
    for (int m = 0; m < P::RMAX; ++m) {
      const int ky = tl + m * T;
      const c2 own = lds0[lds_idx(ky)];
      const c2 w = lds0[lds_idx(ky == 0 ? 0 : N - ky)];
      use(m, own, c2{w.x, -w.y});
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Column kernel of one PAGD iteration.
//
// With q = |k|^2 > 0 and L the averaged-Newton symbol, Lq = q L =
// beta_-2 + theta_l q (beta_0 + beta_2 q + beta_4 q^2), the preconditioned
// residual is
//   d^ = -(1/(P Lq)) [ (a/theta v^ + g^)/M + q mu~^ ],
//   PFC: q mu~^ = q N^ + q (1 - eps - 2q + q^2) v^,
//   FCH: q mu~^ = eps^2 q^2 F'^ + q p^ + q (eps^4 q^2 - eps^2 eta1 q) v^,
// and d^ = 0 at k = 0.  The bracket is accumulated field by field as it
// comes out of its y-transform (the next field's load in flight meanwhile).
//
// One block per column block (cb physical columns of one instance).  The
// instance record is staged in LDS and its scalars are held in scalar
// registers, the field pointers are scalar bases with 32-bit offsets, and
// |k|^2 is recomputed per use from an opaque copy of the thread index
// instead of being held across the transforms: with its twiddles in LDS the
// FCH 2048 plan fits 168 registers per lane (three waves per SIMD, two
// otherwise) and the radix-4 1024 plan 128 (four).
// ---------------------------------------------------------------------------
template <class PY, int MODEL>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(PY::MIN_WAVES))) void k_col_iter(
    const InstDev* const* __restrict__ grp, int bpi, int l, int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  constexpr int NF = MODEL == MODEL_PFC ? 2 : 3;  // transformed fields; the last is v_breve
  const int rows = N;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = uni_i(*I->iter_base + l);
  if (uni_i(stopped_before(I, j))) return;
  const int lbi = uni_i(gpos.lb);
  const ColPos pos = col_pos(T, uni_i(I->nh) / TW, lbi);
  const int t = pos.t, kp = pos.kp;
  c2* lds = smem + pos.c * lds_len(N);
  const bool special = kp == 0;  // this thread's column holds kx = 0 and kx = nx/2
  const bool blk0 = lbi == 0;    // the block holding physical column 0
  const uint32_t fs = (uint32_t)uni_u64((uint64_t)I->field_stride);
  GLB c2* S = gp(uni_p(I->S));
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);

  double bm2, b0, b2, b4;
  betas(I, bm2, b0, b2, b4);
  // the step's first iteration without a column set-up: g^ and the
  // averaged-Newton constants are formed here
  const bool first = uni_i(j == 0 && I->fold_g);
  if (first) fold_betas(I, const_cast<InstDev*>(gpos.I), blk0, b0, b2);
  bm2 = uni_d(bm2);
  b0 = uni_d(b0);
  b2 = uni_d(b2);
  b4 = uni_d(b4);
  const double thl = uni_d(I->theta_l), inv_m = uni_d(I->inv_mobility), aot = uni_d(I->a_over_theta);
  const double inv_p = uni_d(I->inv_p);
  const double kxs = uni_d(I->kx_scale), kys = uni_d(I->ky_scale);
  const double hx = 0.5 * uni_i(I->nx) * kxs;
  const double kxn2 = hx * hx;
  const double kx2 = (kp * kxs) * (kp * kxs);
  auto q_at = [&](int ky) {  // |k|^2 of this thread's logical column (kx = 0 for column 0)
    const double a = (ky <= N / 2 ? ky : ky - N) * kys;
    return kx2 + a * a;
  };
  auto q_col0 = [&](int ky) {  // |k|^2 at kx = 0
    const double a = (ky <= N / 2 ? ky : ky - N) * kys;
    return a * a;
  };
  const double eps = uni_d(I->eps);
  const double e2 = eps * eps, e4 = e2 * e2, e2h1 = e2 * uni_d(I->eta1), e1 = 1.0 - eps;
  auto coef = [&](int f, double q) -> double {
    if (f == NF - 1) {
      const double lin = MODEL == MODEL_PFC ? e1 - 2.0 * q + q * q : e4 * q * q - e2h1 * q;
      return inv_m * aot + q * lin;
    }
    if (MODEL == MODEL_FCH && f == 0) return e2 * q * q;
    return q;
  };
  GLB c2* gsrc = gp(uni_p(first ? I->G : I->ghat));
  GLB c2* ghat = gp(uni_p(I->ghat));
  // scale by -1/(P Lq), zero at k = 0 (without a branch: one inside the
  // unrolled column-0 loops costs spills)
  int bad = 0;
  auto scale = [&](double q) -> double {
    const double Lq = bm2 + thl * q * (b0 + b2 * q + b4 * q * q);
    const bool pos = q > 0.0;
    bad |= pos & !(Lq > 0.0);
    const double r = -inv_p * rcp_pos(Lq);
    return pos ? r : 0.0;
  };
  // Column 0 packs kx = 0 with kx = Nx/2, whose symbols differ by many
  // orders of magnitude at large Nx (eps^4 q^3 at q = (pi/h)^2).  Mixing the
  // packed values with the bracket's symbols and scaling afterwards would
  // recover the kx = 0 part as a difference of terms of the size of the
  // kx = Nx/2 symbol, and the rounding of that difference would set a floor
  // for ||d||_inf.  Column 0 therefore takes the product of symbol and
  // scale per logical column (of moderate size on both), all of it inside
  // the mirror exchange (its own values and their mirror together), and is
  // not scaled again; `keep` is 0 on column 0 and 1 elsewhere.
  auto sig = [&](int f, double q) { return coef(f, q) * scale(q); };
  const double keep = special ? 0.0 : 1.0;

  c2 v[RM], nxt[RM], acc[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    v[m] = gload(S + sidx(rows, t + m * T, kp));
    acc[m] = c2{0.0, 0.0};
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) {
    {
      const int tl = opaque(t);
#pragma unroll
      for (int m = 0; m < RM; ++m)  // prefetch the next field, then g^ (first: g, transformed below)
        nxt[m] = f + 1 < NF ? gload(S + (f + 1) * fs + sidx(rows, tl + m * T, kp))
                            : gload(gsrc + sidx(rows, tl + m * T, kp));
    }
    fft<PY, false>(v, lds, tw, t);
    {
      const int tl = opaque(t);
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        acc[m] = cadd(acc[m], cscale(v[m], keep * coef(f, q_at(tl + m * T))));
      }
    }
    if (blk0)
      col0_pair<PY>(v, smem, special, t, [&](int m, c2 own, c2 w) {
        const double q = q_col0(opaque(t + m * T));
        const double s0 = sig(f, q), sn = sig(f, q + kxn2);
        acc[m] = cadd(acc[m], cadd(cscale(own, 0.5 * (s0 + sn)), cscale(w, 0.5 * (s0 - sn))));
      });
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = nxt[m];
  }
  if (first) {  // g^ for this and the step's later iterations
    fft<PY, false>(v, lds, tw, t);
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) gstore(ghat + sidx(rows, tl + m * T, kp), v[m]);
  }
  // g^ enters with the coefficient 1/M on both logical columns (column 0:
  // times each one's scale, as above)
  {
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = cadd(acc[m], cscale(v[m], keep * inv_m));
  }
  if (blk0)
    col0_pair<PY>(v, smem, special, t, [&](int m, c2 own, c2 w) {
      const double q = q_col0(opaque(t + m * T));
      const double s0 = inv_m * scale(q), sn = inv_m * scale(q + kxn2);
      acc[m] = cadd(acc[m], cadd(cscale(own, 0.5 * (s0 + sn)), cscale(w, 0.5 * (s0 - sn))));
    });
  {
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = special ? acc[m] : cscale(acc[m], scale(q_at(tl + m * T)));
  }
  if constexpr (MODEL == MODEL_FCH) {
    // keep d^ for the Laplacian field: acc <- d^ (packed for column 0)
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = v[m];
  }
  fft<PY, true>(v, lds, tw, t);
  {
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) gstore(S + sidx(rows, tl + m * T, kp), v[m]);
  }
  if constexpr (MODEL == MODEL_FCH) {
    // Delta d: symbol -q on each logical column
    {
      const int tl = opaque(t);
#pragma unroll
      for (int m = 0; m < RM; ++m) v[m] = cscale(acc[m], -q_at(tl + m * T));
    }
    if (blk0)
      col0_mirror<PY>(acc, smem, special, t, [&](int m, c2 w) {
        const double q = q_col0(opaque(t + m * T));
        v[m] = cadd(cscale(acc[m], -(q + 0.5 * kxn2)), cscale(w, 0.5 * kxn2));
      });
    fft<PY, true>(v, lds, tw, t);
    const int tl = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) gstore(S + fs + sidx(rows, tl + m * T, kp), v[m]);
  }
  if (bad) atomicOr(I->flags, FLAG_PRECOND);
}

// ---------------------------------------------------------------------------
// Row kernel of one PAGD iteration (end of j, start of j+1).
// ---------------------------------------------------------------------------
template <class PX>
__device__ __forceinline__ void pair_forward(const double (&a)[PX::RMAX], const double (&b)[PX::RMAX],
                                             const Twiddles<PX>& tw, c2* lds, GLB c2* F, int r0, int rows,
                                             int t) {
  constexpr int RM = PX::RMAX;
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) z[m] = c2{a[m], b[m]};
  fft<PX, false>(z, lds, tw, t);
  unpack_store<PX>(z, lds, F, r0, rows, t);
}

// The forward transforms that start a PFC iteration, for the two real rows
// r0, r0 + 1 of v_breve: field 0 <- (v^3)^, field 1 <- v^.  Rows are paired
// within a field so that each transform writes whole 128-byte lines of the
// tiled spectral layout (two adjacent rows of one tile).
template <class PX>
__device__ __forceinline__ void pfc_forward_pair(const InstDev* I, const double (&vb)[2][PX::RMAX],
                                                 const Twiddles<PX>& tw, c2* lds, int r0, int t) {
  constexpr int RM = PX::RMAX;
  GLB c2* S = gp(uni_p(I->S));
  const uint32_t fs = (uint32_t)uni_u64((uint64_t)I->field_stride);
  const int rows = uni_i(I->rows);
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) z[m] = c2{vb[0][m] * vb[0][m] * vb[0][m], vb[1][m] * vb[1][m] * vb[1][m]};
  fft<PX, false>(z, lds, tw, t);
  unpack_store<PX>(z, lds, S, r0, rows, t);
  pair_forward<PX>(vb[0], vb[1], tw, lds, S + fs, r0, rows, t);
}

// FCH pointwise terms at v_breve with Laplacian lv:
//   F' = (v^2-1)(v+tau), F'' = 3v^2 - 1 + 2 tau v, omega = eps^2 lv - F',
//   p = -F'' omega - eta2 F'.
// Forward transforms for the rows r0, r0 + 1, paired within each field:
// field 0 <- (F')^, field 1 <- p^, field 2 <- v^.
template <class PX>
__device__ __forceinline__ void fch_forward_pair(const InstDev* I, const double (&vb)[2][PX::RMAX],
                                                 const double (&lv)[2][PX::RMAX], const Twiddles<PX>& tw,
                                                 c2* lds, int r0, int t) {
  constexpr int RM = PX::RMAX;
  const double eps = uni_d(I->eps);
  const double e2 = eps * eps, tau = uni_d(I->tau), eta2 = uni_d(I->eta2);
  GLB c2* S = gp(uni_p(I->S));
  const uint32_t fs = (uint32_t)uni_u64((uint64_t)I->field_stride);
  const int rows = uni_i(I->rows);
  c2 z[RM];
  // p first: lv is no longer needed once it is formed.
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    double pr[2];
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      const double u = vb[row][m];
      const double f1 = (u * u - 1.0) * (u + tau);
      const double f2 = 3.0 * u * u - 1.0 + 2.0 * tau * u;
      const double om = e2 * lv[row][m] - f1;
      pr[row] = -f2 * om - eta2 * f1;
    }
    z[m] = c2{pr[0], pr[1]};
  }
  fft<PX, false>(z, lds, tw, t);
  unpack_store<PX>(z, lds, S + fs, r0, rows, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const double u0 = vb[0][m], u1 = vb[1][m];
    z[m] = c2{(u0 * u0 - 1.0) * (u0 + tau), (u1 * u1 - 1.0) * (u1 + tau)};
  }
  fft<PX, false>(z, lds, tw, t);
  unpack_store<PX>(z, lds, S, r0, rows, t);
  pair_forward<PX>(vb[0], vb[1], tw, lds, S + 2 * fs, r0, rows, t);
}

// MPS: implicit midpoint (the nonlinear terms are taken at
// theta y + (1 - theta) u^n); otherwise theta = 1 and u^n is not read.
// The plan's register budget, except for the FCH midpoint form, which holds
// u^n and its Laplacian besides and would spill under it.
template <class PX, int MODEL, bool MPS>
constexpr int row_min_waves() {
  return MODEL == MODEL_FCH && MPS ? 1 : PX::MIN_WAVES;
}

template <class PX, int MODEL, bool MPS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(row_min_waves<PX, MODEL, MPS>()))) void k_row_iter(
    const InstDev* const* __restrict__ grp, int bpi,
                                                  int l, int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ uint64_t red[4];
  __shared__ InstDev rec;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = uni_i(*I->iter_base + l);
  if (uni_i(stopped_before(I, j))) return;
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (gpos.lb * teams + team);
  // record scalars and field bases in scalar registers; element offsets
  // from opaque copies of t, formed where they are used
  const int rows = uni_i(I->rows);
  const uint32_t fs = (uint32_t)uni_u64((uint64_t)I->field_stride);
  const int ne = uni_i(I->n_eta);
  const double lam = uni_d(I->lam[j % ne]), lamn = uni_d(I->lam[(j + 1) % ne]);
  const double s = uni_d(I->s), th = uni_d(I->theta);
  constexpr bool mp = MPS;
  const auto xj = gp(uni_p(I->X[j % 3]));
  const auto xm = gp(uni_p(I->X[(j + 2) % 3]));
  auto xn = gp(uni_p(I->X[(j + 1) % 3]));
  const auto un = gp(uni_p(I->un));
  GLB c2* Sg = gp(uni_p(I->S));
  uint64_t dmax = 0;
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);

  if constexpr (MODEL == MODEL_PFC) {
    double a[2][RM], b[2][RM], uu[2][RM];
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        a[row][m] = xj[idx];
        b[row][m] = xm[idx];
        uu[row][m] = mp ? un[idx] : 0.0;
      }
    }
    c2 v[RM];
    load_pack<PX>(v, Sg, r0, rows, t);
    fft<PX, true>(v, lds, tw, t);
    double vb[2][RM];
    const int tl = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
        const double d = row ? v[m].y : v[m].x;
        const double y = a[row][m] + lam * (a[row][m] - b[row][m]);
        const double x1 = y + s * d;
        xn[idx] = x1;
        const uint64_t db = dbits(fabs(d));
        dmax = db > dmax ? db : dmax;
        const double yn = x1 + lamn * (x1 - a[row][m]);
        vb[row][m] = mp ? th * yn + (1.0 - th) * uu[row][m] : yn;
      }
    }
    pfc_forward_pair<PX>(I, vb, tw, lds, r0, t);
  } else {
    const auto dxj = gp(uni_p(I->DX[j % 3]));
    const auto dxm = gp(uni_p(I->DX[(j + 2) % 3]));
    auto dxn = gp(uni_p(I->DX[(j + 1) % 3]));
    const auto dun = gp(uni_p(I->dun));
    // Both real rows of the pair at once, one transform per spectral field:
    // the direction d (field 0) first, then its Laplacian (field 1), so
    // every spectral read covers whole 128-byte lines of the tiled layout.
    // Large plans issue the real-space loads of each half just before its
    // transform, so that they are in flight during it (226 registers at
    // 2048, two waves per SIMD; the second spectral field is loaded after
    // the first half, which would not fit beside them); small plans
    // (latency-bound grids) issue every load up front.
    constexpr bool EARLY = RM <= 4;
    double vbs[2][RM], lv[2][RM];
    double a[2][RM], b[2][RM], uu[2][RM], la[2][RM], lb[2][RM], lu[2][RM];
    auto load_x = [&]() {
      const int tl = opaque(t);
#pragma unroll
      for (int row = 0; row < 2; ++row) {
#pragma unroll
        for (int m = 0; m < RM; ++m) {
          const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
          a[row][m] = xj[idx];
          b[row][m] = xm[idx];
          uu[row][m] = mp ? un[idx] : 0.0;
        }
      }
    };
    auto load_l = [&]() {
      const int tl = opaque(t);
#pragma unroll
      for (int row = 0; row < 2; ++row) {
#pragma unroll
        for (int m = 0; m < RM; ++m) {
          const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
          la[row][m] = dxj[idx];
          lb[row][m] = dxm[idx];
          lu[row][m] = mp ? dun[idx] : 0.0;
        }
      }
    };
    c2 v[RM], w[RM];
    load_pack<PX>(v, Sg, r0, rows, t);
    if constexpr (EARLY) {
      load_pack<PX>(w, Sg + fs, r0, rows, t);
      load_x();
      load_l();
    }
    if constexpr (!EARLY) load_x();
    fft<PX, true>(v, lds, tw, t);
    const int tx = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tx + m * T;
        const double d = row ? v[m].y : v[m].x;
        const double y = a[row][m] + lam * (a[row][m] - b[row][m]);
        const double x1 = y + s * d;
        xn[idx] = x1;
        const uint64_t db = dbits(fabs(d));
        dmax = db > dmax ? db : dmax;
        const double yn = x1 + lamn * (x1 - a[row][m]);
        vbs[row][m] = mp ? th * yn + (1.0 - th) * uu[row][m] : yn;
      }
    }
    if constexpr (!EARLY) load_pack<PX>(w, Sg + fs, r0, rows, opaque(t));
    if constexpr (!EARLY) load_l();
    fft<PX, true>(w, lds, tw, t);
    const int tw2 = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tw2 + m * T;
        const double ld = row ? w[m].y : w[m].x;
        const double ly = la[row][m] + lam * (la[row][m] - lb[row][m]);
        const double lx1 = ly + s * ld;
        dxn[idx] = lx1;
        const double lyn = lx1 + lamn * (lx1 - la[row][m]);
        lv[row][m] = mp ? th * lyn + (1.0 - th) * lu[row][m] : lyn;
      }
    }
    fch_forward_pair<PX>(I, vbs, lv, tw, lds, r0, t);
  }
  const uint64_t bm = block_max_bits(dmax, red);
  if (threadIdx.x == 0) atomicMax((unsigned long long*)&I->norms[j], (unsigned long long)bm);
}

// ---------------------------------------------------------------------------
// Field-parallel iteration kernels for short transforms, where a kernel's
// time is the latency of its chain of transforms rather than HBM traffic:
// each row pair (column) gets one team of T threads per spectral field (FCH
// three, PFC two), so the transforms of an iteration run side by side
// instead of one after another (FCH rows: d and Delta d inverse, then F', p
// and v forward; PFC rows: d inverse, then v^3 and v forward).  Values cross
// between the teams through LDS.  Same arithmetic as k_row_iter /
// k_col_iter.
// ---------------------------------------------------------------------------
template <int MODEL>
constexpr int fp_teams() { return MODEL == MODEL_FCH ? 3 : 2; }

template <class PX, int MODEL, bool MPS>
__global__ __launch_bounds__(256) void k_row_iter_fp(const InstDev* const* __restrict__ grp, int bpi,
                                                     int l, int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ uint64_t red[4];
  __shared__ InstDev rec;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX, NT = fp_teams<MODEL>();
  constexpr bool fch = MODEL == MODEL_FCH;
  constexpr int NINV = fch ? 2 : 1;              // teams with an inverse transform
  const int npair = blockDim.x / (NT * T);       // row pairs per block
  const int pr = threadIdx.x / (NT * T);         // this thread's pair
  const int role = (threadIdx.x / T) % NT;       // FCH 0: d, F'  1: Delta d, p  2: v;  PFC 0: d, v^3  1: v
  const int t = threadIdx.x % T;
  c2* lds = smem + (pr * NT + role) * lds_len(N);
  // per pair: v_breve of both rows (FCH: then its Laplacian of both rows)
  double* ex = (double*)(smem + npair * NT * lds_len(N) + tw_lds_count<PX>()) + pr * 2 * NINV * N;
  const int r0 = 2 * (gpos.lb * npair + pr);
  const int rows = I->rows;
  const uint32_t fs = (uint32_t)I->field_stride;
  const int ne = I->n_eta;
  const double lam = I->lam[j % ne], lamn = I->lam[(j + 1) % ne];
  const double s = I->s, th = I->theta;
  constexpr bool mp = MPS;
  GLB c2* S = gp(I->S);
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);
  uint64_t dmax = 0;

  // inverse transform of this team's field (the other teams transform zeros)
  c2 v[RM];
  double a[2][RM], b[2][RM], uu[2][RM];
  const GLB double* xa = gp(role == 0 ? I->X[j % 3] : I->DX[j % 3]);
  const GLB double* xb = gp(role == 0 ? I->X[(j + 2) % 3] : I->DX[(j + 2) % 3]);
  const GLB double* xu = gp(role == 0 ? I->un : I->dun);
  if (role < NINV) {
    load_pack<PX>(v, S + role * fs, r0, rows, t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        a[row][m] = xa[idx];
        b[row][m] = xb[idx];
        uu[row][m] = mp ? xu[idx] : 0.0;
      }
    }
  } else {
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = c2{0.0, 0.0};
  }
  fft<PX, true>(v, lds, tw, t);
  if (role < NINV) {
    GLB double* xo = gp(role == 0 ? I->X[(j + 1) % 3] : I->DX[(j + 1) % 3]);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        const double d = row ? v[m].y : v[m].x;
        const double y = a[row][m] + lam * (a[row][m] - b[row][m]);
        const double x1 = y + s * d;
        xo[idx] = x1;
        if (role == 0) {
          const uint64_t db = dbits(fabs(d));
          dmax = db > dmax ? db : dmax;
        }
        const double yn = x1 + lamn * (x1 - a[row][m]);
        ex[(2 * role + row) * N + t + m * T] = mp ? th * yn + (1.0 - th) * uu[row][m] : yn;
      }
    }
  }
  __syncthreads();

  // forward transform of this team's pointwise field
  const double e2 = I->eps * I->eps, tau = I->tau, eta2 = I->eta2;
  c2 z[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    const int k = t + m * T;
    double f[2];
#pragma unroll
    for (int row = 0; row < 2; ++row) {
      const double u = ex[row * N + k];
      if constexpr (fch) {
        const double f1 = (u * u - 1.0) * (u + tau);
        if (role == 0) {
          f[row] = f1;
        } else if (role == 1) {
          const double f2 = 3.0 * u * u - 1.0 + 2.0 * tau * u;
          const double om = e2 * ex[(2 + row) * N + k] - f1;
          f[row] = -f2 * om - eta2 * f1;
        } else {
          f[row] = u;
        }
      } else {
        f[row] = role == 0 ? u * u * u : u;
      }
    }
    z[m] = c2{f[0], f[1]};
  }
  fft<PX, false>(z, lds, tw, t);
  unpack_store<PX>(z, lds, S + role * fs, r0, rows, t);
  const uint64_t bm = block_max_bits(dmax, red);
  if (threadIdx.x == 0) atomicMax((unsigned long long*)&I->norms[j], (unsigned long long)bm);
}

// One column per block, one team per transformed field: forward
// y-transforms side by side, the k-space bracket summed through LDS, then
// the inverse transforms (FCH: d^ and -q d^ side by side).
template <class PY, int MODEL>
__global__ __launch_bounds__(512) void k_col_iter_fp(const InstDev* const* __restrict__ grp, int bpi, int l,
                                                     int /*total*/) {
  extern __shared__ c2 smem[];
  __shared__ InstDev rec;
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = stage_record(gpos.I, &rec);
  const int j = *I->iter_base + l;
  if (stopped_before(I, j)) return;
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX, NT = fp_teams<MODEL>();
  constexpr bool fch = MODEL == MODEL_FCH;
  const int rows = N;
  const int role = threadIdx.x / T, t = threadIdx.x % T;
  // physical column: the tiles' four columns go to blocks lb, lb + 8, ...
  // (same L2 for the partial-line accesses of one tile)
  const int lb = gpos.lb, ntiles = I->nh / TW;
  int tile, sub;
  if ((ntiles & 7) == 0) {
    const int g = lb / (8 * TW), r = lb % (8 * TW);
    tile = g * 8 + (r & 7);
    sub = r >> 3;
  } else {
    tile = lb / TW;
    sub = lb % TW;
  }
  const int kp = tile * TW + sub;
  c2* lds = smem + role * lds_len(N);
  c2* ex = smem + NT * lds_len(N) + tw_lds_count<PY>();  // [NT][N] bracket parts
  const bool special = kp == 0;
  const bool blk0 = lb == 0;
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* S = gp(I->S);
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);
  double bm2, b0, b2, b4;
  betas(I, bm2, b0, b2, b4);
  // the step's first iteration without a column set-up: g^ and the
  // averaged-Newton constants are formed here
  const bool first = j == 0 && I->fold_g;
  if (first) fold_betas(I, const_cast<InstDev*>(gpos.I), blk0, b0, b2);
  // the record's scalars in scalar registers
  bm2 = uni_d(bm2);
  b0 = uni_d(b0);
  b2 = uni_d(b2);
  b4 = uni_d(b4);
  const double thl = uni_d(I->theta_l), inv_m = uni_d(I->inv_mobility), aot = uni_d(I->a_over_theta);
  const double inv_p = uni_d(I->inv_p);
  const double kxs = uni_d(I->kx_scale), kys = uni_d(I->ky_scale);
  const double hx = 0.5 * uni_i(I->nx) * kxs;
  const double kxn2 = hx * hx;
  const double kx2 = (kp * kxs) * (kp * kxs);
  auto q_of = [&](int ky) {
    const double a = (ky <= N / 2 ? ky : ky - N) * kys;
    return kx2 + a * a;
  };
  auto q_col0 = [&](int ky) {
    const double a = (ky <= N / 2 ? ky : ky - N) * kys;
    return a * a;
  };
  const double eps = uni_d(I->eps);
  const double e2 = eps * eps, e4 = e2 * e2, e2h1 = e2 * uni_d(I->eta1), e1 = 1.0 - eps;
  auto coef_f = [&](int f, double q) -> double {
    if (f == NT - 1) {  // v_breve
      const double lin = fch ? e4 * q * q - e2h1 * q : e1 - 2.0 * q + q * q;
      return inv_m * aot + q * lin;
    }
    if (fch && f == 0) return e2 * q * q;
    return q;
  };
  auto coef = [&](double q) { return coef_f(role, q); };
  // scale by -1/(P Lq), zero at k = 0
  int bad = 0;
  auto scale = [&](double q) -> double {
    const double Lq = bm2 + thl * q * (b0 + b2 * q + b4 * q * q);
    const bool pos = q > 0.0;
    bad |= pos & !(Lq > 0.0);
    const double r = -inv_p * rcp_pos(Lq);
    return pos ? r : 0.0;
  };

  c2 v[RM], acc[RM], gh[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = gload(S + role * fs + sidx(rows, t + m * T, kp));
  if (first) {  // g^ = y-transform of the set-up's g rows (every team transforms; the last keeps it)
#pragma unroll
    for (int m = 0; m < RM; ++m)
      gh[m] = role == NT - 1 ? gload(gp(I->G) + sidx(rows, t + m * T, kp)) : c2{0.0, 0.0};
    fft<PY, false>(gh, lds, tw, t);
    if (role == NT - 1) {
#pragma unroll
      for (int m = 0; m < RM; ++m) gstore(gp(I->ghat) + sidx(rows, t + m * T, kp), gh[m]);
    }
  } else if (role == NT - 1) {
#pragma unroll
    for (int m = 0; m < RM; ++m) gh[m] = gload(gp(I->ghat) + sidx(rows, t + m * T, kp));
  }
  fft<PY, false>(v, lds, tw, t);
  {
    const int tf = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = cscale(v[m], coef(q_of(tf + m * T)));
  }
  if (role == NT - 1) {
    // g^ enters with the coefficient 1/M
#pragma unroll
    for (int m = 0; m < RM; ++m) acc[m] = cadd(acc[m], cscale(gh[m], inv_m));
  }
  // Column 0 (kx = 0 and kx = nx/2 packed) keeps its transforms as they are
  // and g^ besides, in the last team's transform buffer once every
  // transform is done; the symbols of the two logical columns differ by
  // orders of magnitude, so each is multiplied by its scale before the two
  // are combined, and the result is not scaled again.
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    c2 x = acc[m];
    if (special) x = v[m];
    ex[role * N + t + m * T] = x;
  }
  if (blk0) {
    __syncthreads();
    if (special && role == NT - 1) {
      const int ts = opaque(t);
#pragma unroll
      for (int m = 0; m < RM; ++m) lds[lds_idx(ts + m * T)] = gh[m];
    }
  }
  __syncthreads();
  if (!special) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int k = t + m * T;
      acc[m] = fch ? cadd(cadd(ex[k], ex[N + k]), ex[2 * N + k]) : cadd(ex[k], ex[N + k]);
    }
  } else {
    const c2* gl = smem + (NT - 1) * lds_len(N);
    const int tc = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int k = tc + m * T, km = k == 0 ? 0 : N - k;
      const double q = q_col0(k);
      const double s0 = scale(q), sn = scale(q + kxn2);
      // c0 F0^ + i cN FN^ = (c0 + cN)/2 P^(ky) + (c0 - cN)/2 conj(P^(-ky))
      auto term = [&](c2 own, c2 mir, double c0, double cn) {
        return cadd(cscale(own, 0.5 * (c0 + cn)), cscale(c2{mir.x, -mir.y}, 0.5 * (c0 - cn)));
      };
      c2 a = term(gl[lds_idx(k)], gl[lds_idx(km)], inv_m * s0, inv_m * sn);
#pragma unroll
      for (int f = 0; f < NT; ++f)
        a = cadd(a, term(ex[f * N + k], ex[f * N + km], coef_f(f, q) * s0, coef_f(f, q + kxn2) * sn));
      acc[m] = a;
    }
  }
  // every team has read g^ from the last team's buffer before any team
  // writes its own buffer again
  if (blk0) __syncthreads();

  {
    const int tf = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) v[m] = special ? acc[m] : cscale(acc[m], scale(q_of(tf + m * T)));
  }
  if constexpr (fch) {
    // team 0 keeps d^, the others take -q d^ (team 2's copy is unused)
    if (role > 0) {
#pragma unroll
      for (int m = 0; m < RM; ++m) acc[m] = v[m];
      const int tf = opaque(t);
#pragma unroll
      for (int m = 0; m < RM; ++m) v[m] = cscale(acc[m], -q_of(tf + m * T));
    }
    if (blk0)
      col0_mirror<PY>(acc, lds, special && role > 0, t, [&](int m, c2 w) {
        const double q = q_col0(opaque(t + m * T));
        v[m] = cadd(cscale(acc[m], -(q + 0.5 * kxn2)), cscale(w, 0.5 * kxn2));
      });
  }
  fft<PY, true>(v, lds, tw, t);
  if (role < (fch ? 2 : 1)) {
    const int ts = opaque(t);
#pragma unroll
    for (int m = 0; m < RM; ++m) gstore(S + role * fs + sidx(rows, ts + m * T, kp), v[m]);
  }
  if (bad) atomicOr(I->flags, FLAG_PRECOND);
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
  double* acc_dst;     // where the chunk graph accepts the solution; null = not accepted there
  // FCH: Laplacians of u^n and u^{n-1} kept from the previous steps (null:
  // Delta x0 comes from transforms), and where the accept keeps Delta u^{n+1}
  const double* lun;
  const double* lunm1;
  double* acc_ldst;
  int32_t fold;        // no column set-up: the first column iteration does its part
  int32_t resid;       // evaluate ||r(x0)||_inf instead of solving (see InstDev::resid)
};

// Up to STEP_ARGS_INLINE instances' arguments travel by value with the
// launch (no host-to-device copy before the set-up); larger groups pass a
// device array.
constexpr int STEP_ARGS_INLINE = 4;
struct StepArgsInline {
  StepArgs a[STEP_ARGS_INLINE];
};

template <class PX, int MODEL>
__global__ __launch_bounds__(256) void k_row_setup(InstDev* const* __restrict__ grp,
                                                   const StepArgs* __restrict__ args, int bpi,
                                                   StepArgsInline inl) {
  extern __shared__ c2 smem[];
  __shared__ double red[4];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  InstDev* __restrict__ I = grp[gi];
  const StepArgs sa = args ? args[gi] : inl.a[gi];
  if (sa.lun) return;  // k_row_setup_lap's instance
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (lb * teams + team);
  const int rows = I->rows;
  const uint32_t fs = (uint32_t)I->field_stride;
  const double th = sa.theta;
  auto x0a = gp(I->X[0]);
  auto x0b = gp(I->X[2]);
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);

  if (lb == 0 && threadIdx.x == 0) {
    I->a = sa.a;
    I->theta = sa.theta;
    I->a_over_theta = sa.a / sa.theta;
    I->un = sa.un;
    I->acc_dst = sa.acc_dst;
    I->acc_ldst = sa.acc_ldst;
    I->lap_hist = sa.lun != nullptr;
    I->fold_g = sa.fold;
    I->resid = sa.resid;
    *I->iter_base = 0;
    *I->flags = 0;
    I->rec->stop_iter = -1;
    I->rec->flags = 0;
    I->rec->norm_bits = 0;
  }
  {  // clear the per-iteration norm slots
    const int nthreads = bpi * blockDim.x;
    for (int i = lb * blockDim.x + threadIdx.x; i < I->max_iter; i += nthreads) I->norms[i] = 0;
  }

  double s0 = 0.0, s1 = 0.0;
  double x0v[2][RM], gv[2][RM], uv[2][RM];
  const double eps = I->eps, tau = I->tau, e2 = eps * eps;
#pragma unroll
  for (int row = 0; row < 2; ++row) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
      const double u = gp(sa.un)[idx], um = gp(sa.unm1)[idx];
      const double x0 = sa.xin ? gp(sa.xin)[idx] : u + sa.rho * (u - um);
      x0a[idx] = x0;
      x0b[idx] = x0;
      x0v[row][m] = x0;
      uv[row][m] = u;
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
    pair_forward<PX>(gv[0], gv[1], tw, lds, gp(I->G), r0, rows, t);
    double vb[2][RM];
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) vb[row][m] = th * x0v[row][m] + (1.0 - th) * uv[row][m];
    }
    pfc_forward_pair<PX>(I, vb, tw, lds, r0, t);
  } else {
    pair_forward<PX>(gv[0], gv[1], tw, lds, gp(I->G), r0, rows, t);
    pair_forward<PX>(x0v[0], x0v[1], tw, lds, gp(I->G) + fs, r0, rows, t);
    if (th != 1.0) pair_forward<PX>(uv[0], uv[1], tw, lds, gp(I->G) + 2 * fs, r0, rows, t);
  }
  const double bs0 = block_sum(s0, red);
  const double bs1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    gp(I->part)[2 * lb] = bs0;
    gp(I->part)[2 * lb + 1] = bs1;
  }
}

// FCH step set-up when the Laplacians of u^n and u^{n-1} were kept by the
// previous accepts (extrapolated guess): Delta is linear, so
// Delta x0 = Delta u^n + rho (Delta u^n - Delta u^{n-1}) needs no transform,
// and the transforms that start iteration 0 are done here; the column set-up
// then transforms g only and the start kernel is not needed.  The guess,
// g, the averaged-Newton partial sums and the published scalars are those of
// k_row_setup (same geometry, same order).
template <class PX>
__global__ __launch_bounds__(256) void k_row_setup_lap(InstDev* const* __restrict__ grp,
                                                       const StepArgs* __restrict__ args, int bpi,
                                                       StepArgsInline inl) {
  extern __shared__ c2 smem[];
  __shared__ double red[4];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  InstDev* __restrict__ I = grp[gi];
  const StepArgs sa = args ? args[gi] : inl.a[gi];
  if (!sa.lun) return;  // k_row_setup's instance
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (lb * teams + team);
  const int rows = I->rows;
  const double th = sa.theta;
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);

  if (lb == 0 && threadIdx.x == 0) {
    I->a = sa.a;
    I->theta = sa.theta;
    I->a_over_theta = sa.a / sa.theta;
    I->un = sa.un;
    I->acc_dst = sa.acc_dst;
    I->acc_ldst = sa.acc_ldst;
    I->lap_hist = 1;
    I->fold_g = sa.fold;
    I->resid = sa.resid;
    *I->iter_base = 0;
    *I->flags = 0;
    I->rec->stop_iter = -1;
    I->rec->flags = 0;
    I->rec->norm_bits = 0;
  }
  {  // clear the per-iteration norm slots
    const int nthreads = bpi * blockDim.x;
    for (int i = lb * blockDim.x + threadIdx.x; i < I->max_iter; i += nthreads) I->norms[i] = 0;
  }

  double s0 = 0.0, s1 = 0.0;
  const double tau = uni_d(I->tau), eps = uni_d(I->eps), e2 = eps * eps;
  const double eta1 = uni_d(I->eta1), eta2 = uni_d(I->eta2);
  const auto un = gp(sa.un), unm1 = gp(sa.unm1);
  {  // g first, alone: u^n and u^{n-1} are read again below (from L2)
    double gv[2][RM];
    const int tl = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
        gv[row][m] = sa.gu * un[idx] + sa.gm * unm1[idx];
      }
    }
    pair_forward<PX>(gv[0], gv[1], tw, lds, gp(I->G), r0, rows, t);
  }
  double vb[2][RM];
  {
    const int tl = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
        const double u = un[idx], um = unm1[idx];
        const double x0 = u + sa.rho * (u - um);
        gp(I->X[0])[idx] = x0;
        gp(I->X[2])[idx] = x0;
        const double v = th * x0 + (1.0 - th) * u;
        vb[row][m] = v;
        const double f1 = (v * v - 1.0) * (v + tau);
        const double f2 = 3.0 * v * v - 1.0 + 2.0 * tau * v;
        const double f3 = 6.0 * v + 2.0 * tau;
        s0 += f2 * f2 - eta2 * f2 + f3 * f1;
        s1 += e2 * f2 - eta1 * e2;
      }
    }
  }
  double lv[2][RM];
  {
    const int tl = opaque(t);
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + tl + m * T;
        const double lu = gp(sa.lun)[idx], lum = gp(sa.lunm1)[idx];
        const double lx0 = lu + sa.rho * (lu - lum);
        gp(I->DX[0])[idx] = lx0;
        gp(I->DX[2])[idx] = lx0;
        if (th != 1.0) gp(I->dun)[idx] = lu;
        lv[row][m] = th * lx0 + (1.0 - th) * lu;
      }
    }
  }
  fch_forward_pair<PX>(I, vb, lv, tw, lds, r0, t);
  const double bs0 = block_sum(s0, red);
  const double bs1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    gp(I->part)[2 * lb] = bs0;
    gp(I->part)[2 * lb + 1] = bs1;
  }
}

// Field-parallel form of k_row_setup_lap for one row pair per block: four
// teams, one per transformed field (0: F', 1: p, 2: v_breve, 3: g), so the
// four forward transforms run side by side.  Team 0 forms x0 and v_breve
// (and the averaged-Newton sums), team 1 Delta x0 and Delta v_breve, team 3
// g; after a block barrier each team builds its field from the shared
// v_breve rows and transforms it.  Same outputs as k_row_setup_lap; one
// partial-sum slot per block.
template <class PX>
__global__ __launch_bounds__(256) void k_row_setup_lap_fp(InstDev* const* __restrict__ grp,
                                                          const StepArgs* __restrict__ args, int bpi,
                                                          StepArgsInline inl) {
  extern __shared__ c2 smem[];
  __shared__ double red[4];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  InstDev* __restrict__ I = grp[gi];
  const StepArgs sa = args ? args[gi] : inl.a[gi];
  if (!sa.lun) return;  // k_row_setup's instance
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX, NT = 4;
  const int role = threadIdx.x / T;
  const int t = threadIdx.x - role * T;
  c2* lds = smem + role * lds_len(N);
  // v_breve of rows r0, r0 + 1, then Delta v_breve of both rows
  double* ex = (double*)(smem + NT * lds_len(N) + tw_lds_count<PX>());
  const int r0 = 2 * lb;
  const int rows = I->rows;
  const uint32_t fs = (uint32_t)I->field_stride;
  const double th = sa.theta;
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);

  if (lb == 0 && threadIdx.x == 0) {
    I->a = sa.a;
    I->theta = sa.theta;
    I->a_over_theta = sa.a / sa.theta;
    I->un = sa.un;
    I->acc_dst = sa.acc_dst;
    I->acc_ldst = sa.acc_ldst;
    I->lap_hist = 1;
    I->fold_g = sa.fold;
    I->resid = sa.resid;
    *I->iter_base = 0;
    *I->flags = 0;
    I->rec->stop_iter = -1;
    I->rec->flags = 0;
    I->rec->norm_bits = 0;
  }
  {  // clear the per-iteration norm slots
    const int nthreads = bpi * blockDim.x;
    for (int i = lb * blockDim.x + threadIdx.x; i < I->max_iter; i += nthreads) I->norms[i] = 0;
  }

  double s0 = 0.0, s1 = 0.0;
  const double tau = I->tau, e2 = I->eps * I->eps, eta2 = I->eta2;
  c2 z[RM];
  if (role == 0) {
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        const double u = gp(sa.un)[idx], um = gp(sa.unm1)[idx];
        const double x0 = u + sa.rho * (u - um);
        gp(I->X[0])[idx] = x0;
        gp(I->X[2])[idx] = x0;
        const double v = th * x0 + (1.0 - th) * u;
        ex[row * N + t + m * T] = v;
        const double f1 = (v * v - 1.0) * (v + tau);
        const double f2 = 3.0 * v * v - 1.0 + 2.0 * tau * v;
        const double f3 = 6.0 * v + 2.0 * tau;
        s0 += f2 * f2 - eta2 * f2 + f3 * f1;
        s1 += e2 * f2 - I->eta1 * e2;
      }
    }
  } else if (role == 1) {
#pragma unroll
    for (int row = 0; row < 2; ++row) {
#pragma unroll
      for (int m = 0; m < RM; ++m) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        const double lu = gp(sa.lun)[idx], lum = gp(sa.lunm1)[idx];
        const double lx0 = lu + sa.rho * (lu - lum);
        gp(I->DX[0])[idx] = lx0;
        gp(I->DX[2])[idx] = lx0;
        if (th != 1.0) gp(I->dun)[idx] = lu;
        ex[(2 + row) * N + t + m * T] = th * lx0 + (1.0 - th) * lu;
      }
    }
  } else if (role == 3) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      double g[2];
#pragma unroll
      for (int row = 0; row < 2; ++row) {
        const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
        g[row] = sa.gu * gp(sa.un)[idx] + sa.gm * gp(sa.unm1)[idx];
      }
      z[m] = c2{g[0], g[1]};
    }
  }
  __syncthreads();
  if (role < 3) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const int k = t + m * T;
      double f[2];
#pragma unroll
      for (int row = 0; row < 2; ++row) {
        const double u = ex[row * N + k];
        const double f1 = (u * u - 1.0) * (u + tau);
        if (role == 0) {
          f[row] = f1;
        } else if (role == 1) {
          const double f2 = 3.0 * u * u - 1.0 + 2.0 * tau * u;
          const double om = e2 * ex[(2 + row) * N + k] - f1;
          f[row] = -f2 * om - eta2 * f1;
        } else {
          f[row] = u;
        }
      }
      z[m] = c2{f[0], f[1]};
    }
  }
  fft<PX, false>(z, lds, tw, t);
  GLB c2* dst = role == 3 ? gp(I->G) : gp(I->S) + role * fs;
  unpack_store<PX>(z, lds, dst, r0, rows, t);
  const double bs0 = block_sum(s0, red);
  const double bs1 = block_sum(s1, red);
  if (threadIdx.x == 0) {
    gp(I->part)[2 * lb] = bs0;
    gp(I->part)[2 * lb + 1] = bs1;
  }
}

// Step setup, column part: g^ (stored for the whole step, column 0 packed
// like every spectral field); FCH also the Laplacians of x0 (and of u^n for
// the midpoint rule) back as spectral rows.  Block 0 sums the averaged-Newton
// partial sums.
template <class PY, int MODEL>
__global__ __launch_bounds__(512) void k_col_setup(InstDev* const* __restrict__ grp, int bpi) {
  extern __shared__ c2 smem[];
  const int gi = blockIdx.x / bpi, lb = blockIdx.x - gi * bpi;
  InstDev* __restrict__ I = grp[gi];
  constexpr int N = PY::N, T = PY::T, RM = PY::RMAX;
  const int rows = N;
  const ColPos pos = col_pos(T, I->nh / TW, lb);
  const int t = pos.t, kp = pos.kp;
  c2* lds = smem + pos.c * lds_len(N);
  const bool special = kp == 0;
  const bool blk0 = lb == 0;
  const uint32_t fs = (uint32_t)I->field_stride;
  GLB c2* G = gp(I->G);
  Twiddles<PY> tw;
  load_twiddles<PY>(tw, I->tw_y, t);
  const double kxn2 = (0.5 * I->nx * I->kx_scale) * (0.5 * I->nx * I->kx_scale);
  if (blk0) finish_betas(I);
  c2 v[RM];
#pragma unroll
  for (int m = 0; m < RM; ++m) v[m] = gload(G + sidx(rows, t + m * T, kp));
  fft<PY, false>(v, lds, tw, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) gstore(gp(I->ghat) + sidx(rows, t + m * T, kp), v[m]);
  if constexpr (MODEL == MODEL_FCH) {
    const int nlap = I->lap_hist ? 0 : I->theta != 1.0 ? 2 : 1;
    for (int f = 1; f <= nlap; ++f) {
#pragma unroll
      for (int m = 0; m < RM; ++m) v[m] = gload(G + f * fs + sidx(rows, t + m * T, kp));
      fft<PY, false>(v, lds, tw, t);
      c2 o[RM];
#pragma unroll
      for (int m = 0; m < RM; ++m) o[m] = cscale(v[m], -wavenum2(I, kp, t + m * T, N) * I->inv_p);
      if (blk0)
        col0_mirror<PY>(v, smem, special, t, [&](int m, c2 w) {
          const double q = wavenum2(I, 0, opaque(t + m * T), N);
          o[m] = cadd(cscale(v[m], -(q + 0.5 * kxn2) * I->inv_p), cscale(w, 0.5 * kxn2 * I->inv_p));
        });
      fft<PY, true>(o, lds, tw, t);
#pragma unroll
      for (int m = 0; m < RM; ++m) gstore(G + f * fs + sidx(rows, t + m * T, kp), o[m]);
    }
  }
}

// FCH step setup, second row part: Laplacians of x0 (and u^n) in real
// space, then the forward transforms that start iteration 0 (y_0 = x_0).
template <class PX>
__global__ __launch_bounds__(256) void k_row_start_fch(const InstDev* const* __restrict__ grp, int bpi) {
  extern __shared__ c2 smem[];
  const GroupPos gpos = group_pos(grp, bpi);
  const InstDev* __restrict__ I = gpos.I;
  if (I->lap_hist) return;  // the row set-up has done this step's part
  constexpr int N = PX::N, T = PX::T, RM = PX::RMAX;
  const int teams = blockDim.x / T;
  const int team = threadIdx.x / T, t = threadIdx.x - team * T;
  c2* lds = smem + team * lds_len(N);
  const int r0 = 2 * (gpos.lb * teams + team);
  const int rows = I->rows;
  const uint32_t fs = (uint32_t)I->field_stride;
  const double th = I->theta;
  const bool mp = th != 1.0;
  Twiddles<PX> tw;
  load_twiddles<PX>(tw, I->tw_x, t);
  double lx[2][RM], lu[2][RM];
  c2 v[RM];
  load_pack<PX>(v, gp(I->G) + fs, r0, rows, t);
  fft<PX, true>(v, lds, tw, t);
#pragma unroll
  for (int m = 0; m < RM; ++m) {
    lx[0][m] = v[m].x;
    lx[1][m] = v[m].y;
    lu[0][m] = 0.0;
    lu[1][m] = 0.0;
  }
  if (mp) {
    load_pack<PX>(v, gp(I->G) + 2 * fs, r0, rows, t);
    fft<PX, true>(v, lds, tw, t);
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      lu[0][m] = v[m].x;
      lu[1][m] = v[m].y;
    }
  }
  double vbs[2][RM], lv[2][RM];
#pragma unroll
  for (int row = 0; row < 2; ++row) {
#pragma unroll
    for (int m = 0; m < RM; ++m) {
      const uint32_t idx = (uint32_t)(r0 + row) * N + t + m * T;
      gp(I->DX[0])[idx] = lx[row][m];
      gp(I->DX[2])[idx] = lx[row][m];
      if (mp) gp(I->dun)[idx] = lu[row][m];
      const double x0 = gp(I->X[0])[idx];
      vbs[row][m] = mp ? th * x0 + (1.0 - th) * gp(I->un)[idx] : x0;
      lv[row][m] = mp ? th * lx[row][m] + (1.0 - th) * lu[row][m] : lx[row][m];
    }
  }
  fch_forward_pair<PX>(I, vbs, lv, tw, lds, r0, t);
}

}  // namespace pfch
