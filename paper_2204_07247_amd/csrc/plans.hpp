// Transform plans (radix schedule per length) and the kernel instantiations
// the host dispatches to, per model and length.
#pragma once
#include "kernels2d.hpp"

namespace pfch {

// ---------------------------------------------------------------------------
// Kernel dispatch per transform length.
// ---------------------------------------------------------------------------
struct RowK {
  const void* iter = nullptr;
  const void* setup = nullptr;
  const void* start_fch = nullptr;
  int T = 0;
  int lds_elems = 0;  // per team
};
struct ColK {
  const void* iter = nullptr;
  const void* setup = nullptr;
  int T = 0;
  int lds_elems = 0;  // per column
};

template <class P, int MODEL>
RowK make_row() {
  RowK k;
  k.iter = (const void*)&k_row_iter<P, MODEL>;
  k.setup = (const void*)&k_row_setup<P, MODEL>;
  if (MODEL == MODEL_FCH) k.start_fch = (const void*)&k_row_start_fch<P>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  return k;
}
template <class P, int MODEL>
ColK make_col() {
  ColK k;
  k.iter = (const void*)&k_col_iter<P, MODEL>;
  k.setup = (const void*)&k_col_setup<P, MODEL>;
  k.T = P::T;
  k.lds_elems = lds_len(P::N);
  return k;
}

using P8 = Plan<8, 8>;
using P16 = Plan<16, 8, 2>;
using P32 = Plan<32, 8, 4>;
using P64 = Plan<64, 8, 8>;
using P128 = Plan<128, 8, 8, 2>;
using P256 = Plan<256, 8, 8, 4>;
using P512 = Plan<512, 8, 8, 8>;
using P1024 = Plan<1024, 8, 8, 4, 4>;
using P2048 = Plan<2048, 8, 8, 8, 4>;

template <int MODEL>
bool row_kernels(int n, RowK& k) {
  switch (n) {
    case 8: k = make_row<P8, MODEL>(); return true;
    case 16: k = make_row<P16, MODEL>(); return true;
    case 32: k = make_row<P32, MODEL>(); return true;
    case 64: k = make_row<P64, MODEL>(); return true;
    case 128: k = make_row<P128, MODEL>(); return true;
    case 256: k = make_row<P256, MODEL>(); return true;
    case 512: k = make_row<P512, MODEL>(); return true;
    case 1024: k = make_row<P1024, MODEL>(); return true;
    case 2048: k = make_row<P2048, MODEL>(); return true;
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
    default: return false;
  }
}

inline bool supported_len(int n) { return n >= 8 && n <= 2048 && (n & (n - 1)) == 0; }

}  // namespace pfch
