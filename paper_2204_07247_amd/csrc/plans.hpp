// Transform plans (radix schedule per length) and the kernel instantiations
// the host dispatches to, per model and length.
#pragma once
#include <vector>

#include "kernels2d.hpp"
#include "kernels3d.hpp"
#include "kernels_rhs.hpp"

namespace pfch {

// ---------------------------------------------------------------------------
// Kernel dispatch per transform length.
// ---------------------------------------------------------------------------
struct RowK {
  const void* iter = nullptr;
  const void* setup = nullptr;
  const void* start_fch = nullptr;
  const void* setup_lap = nullptr;  // FCH set-up from kept Laplacians
  const void* setup_lap_fp = nullptr;  // its field-parallel form (one row pair, four teams per block)
  int setup_fp_elems = 0;              // LDS elements of setup_lap_fp
  const void* rhs_fwd = nullptr;  // R(v) row passes (default plans only)
  const void* rhs_mid = nullptr;  // FCH
  const void* rhs_inv = nullptr;
  int T = 0;           // threads per row pair (three teams for field-parallel kernels)
  int fp = 0;          // field-parallel kernel
  int lds_elems = 0;  // per team
  int tw_elems = 0;   // twiddle table after the teams' buffers
  int radix[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};
struct ColK {
  const void* iter = nullptr;
  const void* setup = nullptr;
  const void* rhs_lap = nullptr;  // R(v) column passes (default plans only): FCH Delta v
  const void* rhs = nullptr;      // R^
  int T = 0;           // threads per column (three teams for field-parallel kernels)
  int fp = 0;          // field-parallel kernel: one column per block
  int lds_elems = 0;  // per column
  int tw_elems = 0;   // twiddle table after the columns' buffers
  int radix[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};

template <class P>
void plan_radices(int* r) {
  for (int p = 0; p < 8; ++p) r[p] = p < P::NPASS ? P::radix(p) : 1;
}

// Plan of the row iteration kernel: P, or P with its twiddles in LDS and a
// register budget for more waves per SIMD (specialised below).  The set-up
// and R(v) row kernels keep P; the LDS reserved for twiddles covers both.
template <class P>
struct RowPlan {
  using type = P;
};
template <class P>
constexpr int row_tw_elems() {
  constexpr int a = tw_lds_count<P>(), b = tw_lds_count<typename RowPlan<P>::type>();
  return a > b ? a : b;
}

template <class P, int MODEL, bool MPS>
RowK make_row() {
  RowK k;
  k.iter = (const void*)&k_row_iter<typename RowPlan<P>::type, MODEL, MPS>;
  k.setup = (const void*)&k_row_setup<P, MODEL>;
  if (MODEL == MODEL_FCH) k.start_fch = (const void*)&k_row_start_fch<P>;
  if (MODEL == MODEL_FCH) k.setup_lap = (const void*)&k_row_setup_lap<P>;
  if constexpr (MODEL == MODEL_FCH && 4 * P::T <= 256 && P::N <= 512) {
    k.setup_lap_fp = (const void*)&k_row_setup_lap_fp<P>;
    k.setup_fp_elems = 4 * lds_len(P::N) + tw_lds_count<P>() + 2 * P::N;  // + 4 real rows
  }
  k.rhs_fwd = (const void*)&k_rhs_row_fwd<P, MODEL>;
  if (MODEL == MODEL_FCH) k.rhs_mid = (const void*)&k_rhs_row_mid<P>;
  k.rhs_inv = (const void*)&k_rhs_row_inv<P>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = row_tw_elems<P>();
  plan_radices<P>(k.radix);
  return k;
}
// Iteration kernel only (setup kernels come from the default plan).
template <class P, int MODEL, bool MPS>
RowK make_row_iter() {
  RowK k;
  k.iter = (const void*)&k_row_iter<typename RowPlan<P>::type, MODEL, MPS>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = row_tw_elems<P>();
  plan_radices<P>(k.radix);
  return k;
}
// Plan of the column iteration kernel: the radix schedule P, with the
// twiddles moved to LDS and a register budget for more waves per SIMD where
// that fits without spilling (specialised below).  The set-up and R(v)
// column kernels keep P itself; the LDS reserved for twiddles covers both.
template <class P>
struct ColPlan {
  using type = P;
};
template <class P>
constexpr int col_tw_elems() {
  constexpr int a = tw_lds_count<P>(), b = tw_lds_count<typename ColPlan<P>::type>();
  return a > b ? a : b;
}

template <class P, int MODEL>
ColK make_col() {
  ColK k;
  k.iter = (const void*)&k_col_iter<typename ColPlan<P>::type, MODEL>;
  k.setup = (const void*)&k_col_setup<P, MODEL>;
  if (MODEL == MODEL_FCH) {
    k.rhs_lap = (const void*)&k_rhs_col<P, MODEL, 1>;
    k.rhs = (const void*)&k_rhs_col<P, MODEL, 2>;
  } else {
    k.rhs = (const void*)&k_rhs_col<P, MODEL, 0>;
  }
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = col_tw_elems<P>();
  plan_radices<P>(k.radix);
  return k;
}
template <class P, int MODEL>
ColK make_col_iter() {
  ColK k;
  k.iter = (const void*)&k_col_iter<typename ColPlan<P>::type, MODEL>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = col_tw_elems<P>();
  plan_radices<P>(k.radix);
  return k;
}

// Default radix schedule per length (radix 8 first, one smaller radix last):
// used by the step-setup kernels always and by the iteration kernels unless
// the autotuner picks an alternative.
using P8 = Plan<8, 8>;
using P16 = Plan<16, 8, 2>;
using P32 = Plan<32, 8, 4>;
using P64 = Plan<64, 8, 8>;
using P128 = Plan<128, 8, 8, 2>;
using P256 = Plan<256, 8, 8, 4>;
using P512 = Plan<512, 8, 8, 8>;
using P1024 = Plan<1024, 8, 8, 4, 4>;
using P2048 = Plan<2048, 8, 8, 8, 4>;
using P192 = Plan<192, 3, 4, 4, 4>;  // 12 elements per thread
// FCH 2048 (three transformed fields, eight elements per thread): 158
// registers, three waves per SIMD, with the twiddles in LDS.  (The 2048 row
// kernel is left as it is, 201 registers and two waves: with its twiddles
// in LDS it ran 4% slower, and held to three waves per SIMD with them it
// spills 7 registers and ran 1.4% slower.)
template <>
struct ColPlan<P2048> {
  using type = LdsTw<P2048, 3>;
};

template <int MODEL, bool MPS>
bool row_kernels(int n, RowK& k) {
  switch (n) {
    case 8: k = make_row<P8, MODEL, MPS>(); return true;
    case 16: k = make_row<P16, MODEL, MPS>(); return true;
    case 32: k = make_row<P32, MODEL, MPS>(); return true;
    case 64: k = make_row<P64, MODEL, MPS>(); return true;
    case 128: k = make_row<P128, MODEL, MPS>(); return true;
    case 256: k = make_row<P256, MODEL, MPS>(); return true;
    case 512: k = make_row<P512, MODEL, MPS>(); return true;
    case 1024: k = make_row<P1024, MODEL, MPS>(); return true;
    case 2048: k = make_row<P2048, MODEL, MPS>(); return true;
    case 192: k = make_row<P192, MODEL, MPS>(); return true;
    default: return false;
  }
}
template <int MODEL>
bool col_kernels(int n, ColK& k) {
  switch (n) {
    case 8: k = make_col<P8, MODEL>(); return true;
    case 16: k = make_col<P16, MODEL>(); return true;
    case 32: k = make_col<P32, MODEL>(); return true;
    case 64: k = make_col<P64, MODEL>(); return true;
    case 128: k = make_col<P128, MODEL>(); return true;
    case 256: k = make_col<P256, MODEL>(); return true;
    case 512: k = make_col<P512, MODEL>(); return true;
    case 1024: k = make_col<P1024, MODEL>(); return true;
    case 2048: k = make_col<P2048, MODEL>(); return true;
    case 192: k = make_col<P192, MODEL>(); return true;
    default: return false;
  }
}

// Alternative radix schedules the autotuner may pick for the iteration
// kernels: radix 4 (fewer registers per thread, more threads and passes) and
// radix 16 (fewer passes through LDS, more registers).
using A64a = Plan<64, 4, 4, 4>;
using A64b = Plan<64, 16, 4>;
using A128a = Plan<128, 4, 4, 4, 2>;
using A128b = Plan<128, 16, 8>;
using A256a = Plan<256, 4, 4, 4, 4>;
using A256b = Plan<256, 16, 16>;
using A512a = Plan<512, 16, 16, 2>;
using A1024a = Plan<1024, 16, 16, 4>;
using A1024b = Plan<1024, 4, 4, 4, 4, 4>;
using A2048a = Plan<2048, 16, 16, 8>;
using A192a = Plan<192, 3, 2, 2, 2, 2, 2, 2>;  // 6 elements per thread
// radix 4 at 1024 (four elements per thread): 128 registers, four waves per SIMD
template <>
struct ColPlan<A1024b> {
  using type = LdsTw<A1024b, 4>;
};
// (rows: 84-127 registers with the twiddles in LDS, four or five waves)
template <>
struct RowPlan<A1024b> {
  using type = LdsTw<A1024b, 1>;
};
#define PFCH_ALT_PLANS(X)                                                                          \
  X(64, A64a) X(64, A64b) X(128, A128a) X(128, A128b) X(256, A256a) X(256, A256b) X(512, A512a)   \
  X(1024, A1024a) X(1024, A1024b) X(2048, A2048a) X(192, A192a)

template <int MODEL, bool MPS>
void row_alternatives(int n, std::vector<RowK>& out) {
#define PFCH_ROW_ALT(LEN, PLAN) \
  if (n == LEN) out.push_back(make_row_iter<PLAN, MODEL, MPS>());
  PFCH_ALT_PLANS(PFCH_ROW_ALT)
#undef PFCH_ROW_ALT
}
// Column kernels keep three fields' transforms and the k-space bracket live
// at once; with radix 16 they spill hundreds of bytes per lane, so only the
// radix-4 (and 192's radix-3/2) schedules are column candidates.
#define PFCH_COL_ALT_PLANS(X) X(64, A64a) X(128, A128a) X(256, A256a) X(1024, A1024b) X(192, A192a)
template <int MODEL>
void col_alternatives(int n, std::vector<ColK>& out) {
#define PFCH_COL_ALT(LEN, PLAN) \
  if (n == LEN) out.push_back(make_col_iter<PLAN, MODEL>());
  PFCH_COL_ALT_PLANS(PFCH_COL_ALT)
#undef PFCH_COL_ALT
}

// Field-parallel iteration kernels (one team per spectral field and row pair
// or column) for the lengths where a plan's team is small enough.
template <class P, int MODEL, bool MPS>
RowK make_row_fp() {
  constexpr int NT = fp_teams<MODEL>(), NINV = MODEL == MODEL_FCH ? 2 : 1;
  RowK k;
  k.iter = (const void*)&k_row_iter_fp<P, MODEL, MPS>;
  k.T = NT * P::T;
  k.lds_elems = NT * lds_len(P::N) + NINV * P::N;  // transforms + v_breve (, Delta v_breve) of two rows
  k.tw_elems = tw_lds_count<P>();
  k.fp = 1;
  plan_radices<P>(k.radix);
  return k;
}
template <class P, int MODEL>
ColK make_col_fp() {
  constexpr int NT = fp_teams<MODEL>();
  ColK k;
  k.iter = (const void*)&k_col_iter_fp<P, MODEL>;
  k.T = NT * P::T;
  k.lds_elems = NT * lds_len(P::N) + NT * P::N;  // transforms + the bracket's parts
  k.tw_elems = tw_lds_count<P>();
  k.fp = 1;
  plan_radices<P>(k.radix);
  return k;
}
#define PFCH_FP_PLANS(X) \
  X(64, P64) X(64, A64a) X(128, P128) X(128, A128a) X(256, P256) X(256, A256a) X(512, P512) X(1024, P1024) \
  X(1024, A1024b)

template <int MODEL, bool MPS>
void row_fp_alternatives(int n, std::vector<RowK>& out) {
#define PFCH_ROW_FP(LEN, PLAN) \
  if constexpr (fp_teams<MODEL>() * PLAN::T <= 256) if (n == LEN) out.push_back(make_row_fp<PLAN, MODEL, MPS>());
  PFCH_FP_PLANS(PFCH_ROW_FP)
#undef PFCH_ROW_FP
}
template <int MODEL>
void col_fp_alternatives(int n, std::vector<ColK>& out) {
#define PFCH_COL_FP(LEN, PLAN) \
  if constexpr (fp_teams<MODEL>() * PLAN::T <= 512) if (n == LEN) out.push_back(make_col_fp<PLAN, MODEL>());
  PFCH_FP_PLANS(PFCH_COL_FP)
#undef PFCH_COL_FP
}

// Three-dimensional PFC: kernels of the y- and z-passes per length.
struct Y3K {
  const void* fwd = nullptr;
  const void* inv = nullptr;
  const void* setup = nullptr;
  const void* rhs_fwd = nullptr;  // R(v) y-passes
  const void* rhs_inv = nullptr;
  int T = 0;
  int lds_elems = 0;
  int tw_elems = 0;
  int radix[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};
struct Z3K {
  const void* iter = nullptr;
  const void* setup = nullptr;
  const void* rhs = nullptr;  // R(v) z-pass
  int T = 0;
  int lds_elems = 0;
  int tw_elems = 0;
  int radix[8] = {1, 1, 1, 1, 1, 1, 1, 1};
};
template <class P>
Y3K make_y3() {
  Y3K k;
  k.fwd = (const void*)&k_y3_iter<P, false>;
  k.inv = (const void*)&k_y3_iter<P, true>;
  k.setup = (const void*)&k_y3_setup<P>;
  k.rhs_fwd = (const void*)&k_rhs_y3<P, false>;
  k.rhs_inv = (const void*)&k_rhs_y3<P, true>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = tw_lds_count<P>();
  plan_radices<P>(k.radix);
  return k;
}
template <class P>
Z3K make_z3() {
  Z3K k;
  k.iter = (const void*)&k_z3_iter<P>;
  k.setup = (const void*)&k_z3_setup<P>;
  k.rhs = (const void*)&k_rhs_z3<P>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  k.tw_elems = tw_lds_count<P>();
  plan_radices<P>(k.radix);
  return k;
}
// y and z lengths of the 3D path
inline bool supported_len3(int n) { return n == 8 || n == 16 || n == 32 || n == 64 || n == 128 || n == 192 || n == 256; }
inline void y3_alternatives(int n, std::vector<Y3K>& out) {
  if (n == 192) out.push_back(make_y3<A192a>());
}
inline void z3_alternatives(int n, std::vector<Z3K>& out) {
  if (n == 192) out.push_back(make_z3<A192a>());
}
inline bool y3_kernels(int n, Y3K& k) {
  switch (n) {
    case 8: k = make_y3<P8>(); return true;
    case 16: k = make_y3<P16>(); return true;
    case 32: k = make_y3<P32>(); return true;
    case 64: k = make_y3<P64>(); return true;
    case 128: k = make_y3<P128>(); return true;
    case 192: k = make_y3<P192>(); return true;
    case 256: k = make_y3<P256>(); return true;
    default: return false;
  }
}
inline bool z3_kernels(int n, Z3K& k) {
  switch (n) {
    case 8: k = make_z3<P8>(); return true;
    case 16: k = make_z3<P16>(); return true;
    case 32: k = make_z3<P32>(); return true;
    case 64: k = make_z3<P64>(); return true;
    case 128: k = make_z3<P128>(); return true;
    case 192: k = make_z3<P192>(); return true;
    case 256: k = make_z3<P256>(); return true;
    default: return false;
  }
}

inline bool supported_len(int n) { return (n >= 8 && n <= 2048 && (n & (n - 1)) == 0) || n == 192; }

}  // namespace pfch
