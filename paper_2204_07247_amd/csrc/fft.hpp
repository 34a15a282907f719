// FP64 complex FFT building blocks for gfx950: register radix-2/3/4/8/16
// butterflies and LDS-staged Stockham autosort passes.
//
// A transform of length N is carried out by a "team" of T = N / RMAX
// threads.  Team thread t owns the elements k = t + m*T, m = 0..RMAX-1, both
// on input (natural order, held in registers v[m]) and on output (natural
// order, again in v[m]).  Between passes the data lives in LDS; the first
// pass reads registers and the last pass writes registers, so a plan of P
// passes costs P-1 LDS round trips.
//
// Pass with radix R after earlier passes of total length Ns (Stockham):
//   butterfly j in [0, N/R) reads  x[j + r*N/R], r = 0..R-1,
//   multiplies input r by w_N^{(j mod Ns) * r * N/(Ns*R)},  w_N = exp(-2 pi i/N),
//   applies the R-point DFT and writes y[(j/Ns)*Ns*R + (j mod Ns) + r*Ns].
// Thread t processes the butterflies j = t + q*T, q = 0..RMAX/R-1.
//
// Twiddles come from a per-length table tw[k] = exp(-2 pi i k / N) computed
// on the host in long double, read once per kernel into registers or, for
// plans that would need many per thread, into an LDS table (Twiddles).
// Inverse transforms use conjugates.  Neither direction is normalised.
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

namespace pfch {

// Device pointers kept in memory are generic; kernels cast them to the
// global address space so that accesses compile to global_load/store
// (generic "flat" accesses also count against the LDS wait counter, which
// every LDS barrier drains).
#define GLB __attribute__((address_space(1)))
template <class T>
__device__ __forceinline__ GLB T* gp(T* p) {
  return (GLB T*)p;
}
template <class T>
__device__ __forceinline__ const GLB T* gp(const T* p) {
  return (const GLB T*)p;
}

struct alignas(16) c2 {
  double x, y;
};

// 16-byte loads and stores of complex values through global pointers.
typedef double f64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ c2 gload(const GLB c2* p) {
  const f64x2 v = *(const GLB f64x2*)p;
  return c2{v.x, v.y};
}
__device__ __forceinline__ void gstore(GLB c2* p, c2 a) {
  f64x2 v;
  v.x = a.x;
  v.y = a.y;
  *(GLB f64x2*)p = v;
}

__device__ __forceinline__ c2 cadd(c2 a, c2 b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ c2 csub(c2 a, c2 b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ c2 cmul(c2 a, c2 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ c2 cconj(c2 a) { return {a.x, -a.y}; }

// 1/x for positive normal x: hardware reciprocal estimate refined by two
// Newton steps (relative error below one ulp); avoids the long IEEE
// division sequence and its register footprint.
__device__ __forceinline__ double rcp_pos(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ c2 cscale(c2 a, double s) { return {a.x * s, a.y * s}; }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ c2 mul_mi(c2 a) {
  return INV ? c2{-a.y, a.x} : c2{a.y, -a.x};
}

// ---------------------------------------------------------------------------
// Small DFTs in registers.  Forward: X[k] = sum_n x[n] exp(-2 pi i n k / R).
// ---------------------------------------------------------------------------
template <bool INV>
__device__ __forceinline__ void dft2(c2& a, c2& b) {
  c2 t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV>
__device__ __forceinline__ void dft3(c2* x) {
  constexpr double H = 0.86602540378443864676372317075294;  // sqrt(3)/2
  c2 t1 = cadd(x[1], x[2]);
  c2 t2 = csub(x[1], x[2]);
  c2 m = {x[0].x - 0.5 * t1.x, x[0].y - 0.5 * t1.y};
  x[0] = cadd(x[0], t1);
  // forward: X1 = m - i H t2, X2 = m + i H t2
  c2 s = mul_mi<INV>(cscale(t2, H));
  x[1] = cadd(m, s);
  x[2] = csub(m, s);
}

template <bool INV>
__device__ __forceinline__ void dft4(c2* x) {
  c2 a0 = cadd(x[0], x[2]);
  c2 a1 = csub(x[0], x[2]);
  c2 b0 = cadd(x[1], x[3]);
  c2 b1 = mul_mi<INV>(csub(x[1], x[3]));
  x[0] = cadd(a0, b0);
  x[2] = csub(a0, b0);
  x[1] = cadd(a1, b1);
  x[3] = csub(a1, b1);
}

template <bool INV>
__device__ __forceinline__ void dft8(c2* x) {
  constexpr double R = 0.70710678118654752440084436210485;  // sqrt(1/2)
  c2 e[4] = {x[0], x[2], x[4], x[6]};
  c2 o[4] = {x[1], x[3], x[5], x[7]};
  dft4<INV>(e);
  dft4<INV>(o);
  // twiddles w8^k, k = 0..3 (forward w8 = exp(-i pi/4))
  const double sg = INV ? 1.0 : -1.0;
  c2 w1 = {R, sg * R}, w3 = {-R, sg * R};
  o[1] = cmul(o[1], w1);
  o[2] = mul_mi<INV>(o[2]);
  o[3] = cmul(o[3], w3);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    x[k] = cadd(e[k], o[k]);
    x[k + 4] = csub(e[k], o[k]);
  }
}

template <bool INV>
__device__ __forceinline__ void dft16(c2* x) {
  constexpr double C1 = 0.92387953251128675612818318939679;  // cos(pi/8)
  constexpr double S1 = 0.38268343236508977172845998403040;  // sin(pi/8)
  constexpr double R = 0.70710678118654752440084436210485;
  c2 e[8], o[8];
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    e[n] = x[2 * n];
    o[n] = x[2 * n + 1];
  }
  dft8<INV>(e);
  dft8<INV>(o);
  const double sg = INV ? 1.0 : -1.0;
  // w16^k = cos(k pi/8) + sg i sin(k pi/8)
  const c2 w[8] = {{1.0, 0.0},      {C1, sg * S1},   {R, sg * R},     {S1, sg * C1},
                   {0.0, sg * 1.0}, {-S1, sg * C1},  {-R, sg * R},    {-C1, sg * S1}};
#pragma unroll
  for (int k = 1; k < 8; ++k) o[k] = cmul(o[k], w[k]);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    x[k] = cadd(e[k], o[k]);
    x[k + 8] = csub(e[k], o[k]);
  }
}

template <int R, bool INV>
__device__ __forceinline__ void dft(c2* x) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    dft2<INV>(x[0], x[1]);
  } else if constexpr (R == 3) {
    dft3<INV>(x);
  } else if constexpr (R == 4) {
    dft4<INV>(x);
  } else if constexpr (R == 8) {
    dft8<INV>(x);
  } else if constexpr (R == 16) {
    dft16<INV>(x);
  } else {
    static_assert(R == 16, "unsupported radix");
  }
}

// LDS index with one pad element per 2^PFCH_LDS_PAD_SHIFT to break
// power-of-two strides.
#ifndef PFCH_LDS_PAD_SHIFT
#define PFCH_LDS_PAD_SHIFT 4
#endif
__device__ __forceinline__ int lds_idx(int i) { return i + (i >> PFCH_LDS_PAD_SHIFT); }
__host__ __device__ constexpr int lds_len(int n) { return n + (n >> PFCH_LDS_PAD_SHIFT) + 1; }

constexpr int cgcd(int a, int b) { return b == 0 ? a : cgcd(b, a % b); }
constexpr int clcm(int a, int b) { return a / cgcd(a, b) * b; }

// Plan: the radices of the passes, first to last.  Each thread holds
// RMAX = lcm of the radices elements, so that it handles whole butterflies
// in every pass (RMAX = 12 for mixed radix 3 and 4).
template <int N_, int... Rs>
struct Plan {
  static constexpr int N = N_;
  static constexpr int NPASS = sizeof...(Rs);
  static constexpr int RS[NPASS] = {Rs...};
  static constexpr int RMAX = [] {
    int l = 1;
    for (int r : RS) l = clcm(l, r);
    return l;
  }();
  static constexpr int T = N / RMAX;
  static constexpr int radix(int p) { return RS[p]; }
  static constexpr int ns(int p) {
    int s = 1;
    for (int i = 0; i < p; ++i) s *= RS[i];
    return s;
  }
  static_assert(NPASS >= 1 && NPASS <= 8, "one to eight passes");
  static_assert(ns(NPASS) == N, "radices must multiply to N");
  static constexpr bool TW_LDS = false;  // twiddles in the LDS table whatever their count
  static constexpr int MIN_WAVES = 1;    // waves per SIMD a kernel of this plan may ask the compiler for
};

// The same radix schedule with its twiddles in the LDS table (freeing the
// registers that hold them) and a kernel register budget for at least
// MINW waves per SIMD.
template <class P, int MINW>
struct LdsTw : P {
  static constexpr bool TW_LDS = true;
  static constexpr int MIN_WAVES = MINW;
};

// Twiddles live in LDS, after the block's transform buffers: for every pass
// p >= 1 the Ns(p) values w_N^{i N/(Ns R)}, i < Ns(p), which are all the
// first-power twiddles w1 = w_N^{(j mod Ns) N/(Ns R)} its butterflies need
// (pass 0 needs none); the powers w1^r are formed by repeated complex
// multiplication (at most 15 products, error a few ulps).  The block fills the
// table once per kernel from the host-computed table of N entries.
template <class P>
constexpr int tw_offset(int p) {  // start of pass p's entries
  int o = 0;
  for (int q = 1; q < p; ++q) o += P::ns(q);
  return o;
}
template <class P>
constexpr int tw_count() {
  return tw_offset<P>(P::NPASS);
}

// Where a plan keeps its twiddles: in registers (each thread holds the
// first powers of its own butterflies, read once per kernel) when that is at
// most four complex values per thread, else in the LDS table (radix-3/2 and
// many-pass plans, whose register copies would cost occupancy).
template <class P>
constexpr int tw_per_thread() {
  int n = 0;
  for (int p = 1; p < P::NPASS; ++p) n += P::RMAX / P::radix(p);
  return n;
}
template <class P>
constexpr bool tw_in_lds() {
  return P::TW_LDS || tw_per_thread<P>() > 4;
}
// LDS entries the plan's twiddle table needs (0 in register mode).
template <class P>
constexpr int tw_lds_count() {
  return tw_in_lds<P>() ? tw_count<P>() : 0;
}

template <class P>
struct Twiddles {
  const c2* lds;                                   // LDS mode
  c2 w[P::NPASS > 1 ? P::NPASS - 1 : 1][P::RMAX];  // register mode
};

// Index into the host table of compact entry i.
template <class P>
__device__ __forceinline__ int tw_source(int i) {
  int p = 1, o = 0;
  while (p + 1 < P::NPASS && i >= o + P::ns(p)) {
    o += P::ns(p);
    ++p;
  }
  return (i - o) * (P::N / (P::ns(p) * P::radix(p)));
}

// Two-phase set-up, so that a kernel can issue its data loads between the
// two.  LDS mode: tw_fetch reads this thread's share of the table into
// registers (blocks have at least T threads, hence the bound) and tw_commit
// stores it into LDS and synchronises the block.  Register mode: tw_fetch
// reads the thread's own twiddles and tw_commit only hands them over.
// Every thread of the block calls tw_commit.
template <class P>
struct TwFetch {
  static constexpr int NT = tw_count<P>();
  static constexpr int PER = tw_in_lds<P>() && NT > 0 ? (NT + P::T - 1) / P::T : 1;
  c2 v[PER];
  c2 w[P::NPASS > 1 ? P::NPASS - 1 : 1][P::RMAX];
};
template <class P>
__device__ __forceinline__ void tw_fetch(TwFetch<P>& f, const c2* __restrict__ table_, int t) {
  const GLB c2* table = gp(table_);
  if constexpr (tw_in_lds<P>()) {
#pragma unroll
    for (int q = 0; q < TwFetch<P>::PER; ++q) {
      const int i = threadIdx.x + q * blockDim.x;
      if (i < TwFetch<P>::NT) f.v[q] = gload(table + tw_source<P>(i));
    }
  } else {
#pragma unroll
    for (int p = 1; p < P::NPASS; ++p) {
      const int R = P::radix(p), NS = P::ns(p), QN = P::RMAX / R;
#pragma unroll
      for (int q = 0; q < P::RMAX; ++q) {
        if (q < QN) {
          const int j = t + q * P::T;
          f.w[p - 1][q] = gload(table + (j % NS) * (P::N / (NS * R)));
        }
      }
    }
  }
}
template <class P>
__device__ __forceinline__ void tw_commit(Twiddles<P>& tw, const TwFetch<P>& f) {
  if constexpr (tw_in_lds<P>()) {
    extern __shared__ c2 smem_tw[];
    c2* dst = smem_tw + (blockDim.x / P::T) * lds_len(P::N);
#pragma unroll
    for (int q = 0; q < TwFetch<P>::PER; ++q) {
      const int i = threadIdx.x + q * blockDim.x;
      if (i < TwFetch<P>::NT) dst[i] = f.v[q];
    }
    __syncthreads();
    tw.lds = dst;
  } else {
#pragma unroll
    for (int p = 1; p < P::NPASS; ++p)
#pragma unroll
      for (int q = 0; q < P::RMAX / P::radix(p); ++q) tw.w[p - 1][q] = f.w[p - 1][q];
  }
}

// Both phases at once.  Every thread of the block calls this.
template <class P>
__device__ __forceinline__ void load_twiddles(Twiddles<P>& tw, const c2* __restrict__ table, int t) {
  TwFetch<P> f;
  tw_fetch<P>(f, table, t);
  tw_commit<P>(tw, f);
}

// One Stockham pass.  FROM_REG / TO_REG select registers or LDS as source
// and destination.  `lds` is the team's buffer of lds_len(N) elements.
template <class P, int PASS, bool INV, bool FROM_REG, bool TO_REG>
__device__ __forceinline__ void stockham_pass(c2 (&v)[P::RMAX], c2* lds, const Twiddles<P>& tw, int t) {
  constexpr int N = P::N, T = P::T, RMAX = P::RMAX;
  constexpr int R = P::radix(PASS);
  constexpr int NS = P::ns(PASS);
  constexpr int QN = RMAX / R;  // butterflies per thread
  constexpr int STRIDE = N / R;
  c2 x[RMAX];
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int j = t + q * T;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if constexpr (FROM_REG) {
        x[q * R + r] = v[q + r * QN];
      } else {
        x[q * R + r] = lds[lds_idx(j + r * STRIDE)];
      }
    }
  }
  if constexpr (!FROM_REG && !TO_REG) __syncthreads();  // all reads before in-place writes
#pragma unroll
  for (int q = 0; q < QN; ++q) {
    const int j = t + q * T;
    if constexpr (NS > 1) {
      c2 w1;
      if constexpr (tw_in_lds<P>())
        w1 = tw.lds[tw_offset<P>(PASS) + j % NS];
      else
        w1 = tw.w[PASS - 1][q];
      if (INV) w1.y = -w1.y;
      c2 w = w1;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        x[q * R + r] = cmul(x[q * R + r], w);
        if (r + 1 < R) w = cmul(w, w1);
      }
    }
    dft<R, INV>(&x[q * R]);
    if constexpr (TO_REG) {
      // last pass: outputs at j + r*N/R, i.e. register q + r*QN
#pragma unroll
      for (int r = 0; r < R; ++r) v[q + r * QN] = x[q * R + r];
    } else {
      const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lds_idx(base + r * NS)] = x[q * R + r];
    }
  }
}

// Opaque copies: the compiler may not merge work that depends on them
// across transforms.  Without this, the twiddle powers and LDS addresses of
// every transform in a kernel are computed once and kept live across all
// barriers, which costs more registers than recomputing them.
__device__ __forceinline__ int opaque_i(int v) {
  asm volatile("" : "+v"(v));
  return v;
}
__device__ __forceinline__ double opaque_d(double v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Passes 1 .. NPASS-2, LDS to LDS.
template <class P, bool INV, int... I>
__device__ __forceinline__ void mid_passes(c2 (&v)[P::RMAX], c2* lds, const Twiddles<P>& tw, int t,
                                           std::integer_sequence<int, I...>) {
  ((stockham_pass<P, I + 1, INV, false, false>(v, lds, tw, t), __syncthreads()), ...);
}

// Full transform: registers in, registers out.  Every thread of the block
// must call this (it contains block-wide barriers when NPASS > 1).
template <class P, bool INV>
__device__ __forceinline__ void fft(c2 (&v)[P::RMAX], c2* lds, const Twiddles<P>& tw_in, int t_in) {
  const int t = opaque_i(t_in);
  Twiddles<P> tw;
  if constexpr (tw_in_lds<P>()) {
    tw.lds = tw_in.lds;
  } else {
#pragma unroll
    for (int p = 1; p < P::NPASS; ++p) {
#pragma unroll
      for (int q = 0; q < P::RMAX / P::radix(p); ++q) {
        tw.w[p - 1][q].x = opaque_d(tw_in.w[p - 1][q].x);
        tw.w[p - 1][q].y = opaque_d(tw_in.w[p - 1][q].y);
      }
    }
  }
  if constexpr (P::NPASS == 1) {
    stockham_pass<P, 0, INV, true, true>(v, lds, tw, t);
  } else {
    stockham_pass<P, 0, INV, true, false>(v, lds, tw, t);
    __syncthreads();
    mid_passes<P, INV>(v, lds, tw, t, std::make_integer_sequence<int, P::NPASS - 2>{});
    stockham_pass<P, P::NPASS - 1, INV, false, true>(v, lds, tw, t);
    __syncthreads();  // LDS free for reuse on return
  }
}

}  // namespace pfch
