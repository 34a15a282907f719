// Host runtime of libpfch: context, workspaces, launch graphs and the C ABI.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "../../include/pfch.h"
#include "kernels2d.hpp"

using namespace pfch;

namespace {

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

bool supported_len(int n) {
  return n >= 8 && n <= 2048 && (n & (n - 1)) == 0;
}

// ---------------------------------------------------------------------------
// Small kernels: end of a chunk of iterations, accept, mass reduction.
// ---------------------------------------------------------------------------
__global__ void k_chunk_end(InstDev* const* insts, int n, int K) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  InstDev* I = insts[i];
  StopRec* rec = I->rec;
  const int base = *I->iter_base;
  if (rec->stop_iter < 0 && base < I->max_iter + 1) {
    for (int jj = base; jj < base + K; ++jj) {
      if (jj >= I->max_iter) {
        rec->stop_iter = I->max_iter;
        rec->norm_bits = I->norms[I->max_iter - 1];
        break;
      }
      const uint64_t b = I->norms[jj];
      if (b < I->tol_bits || b >= INF_BITS) {
        rec->stop_iter = jj;
        rec->norm_bits = b;
        break;
      }
    }
  }
  rec->flags |= *I->flags;
  const bool stop = rec->stop_iter >= 0 || (rec->flags & FLAG_PRECOND);
  *I->iter_base = stop ? I->max_iter + 1 : base + K;
}

constexpr int ACC_BLOCKS = 256, ACC_THREADS = 256;

__global__ __launch_bounds__(ACC_THREADS) void k_copy_sum(const double* __restrict__ src,
                                                          double* __restrict__ dst, int64_t n,
                                                          double* __restrict__ part) {
  __shared__ double red[ACC_THREADS / 64];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = src[i];
    if (dst) dst[i] = v;
    s += v;
  }
  const double b = block_sum(s, red);
  if (threadIdx.x == 0 && part) part[blockIdx.x] = b;
}

__global__ void k_sum_parts(const double* __restrict__ part, int n, double scale, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += part[i];
    *out = s * scale;
  }
}

// ---------------------------------------------------------------------------
// Host structures.
// ---------------------------------------------------------------------------
#define HIPCHK(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return PFCH_E_HIP; \
  } while (0)

struct Instance {
  pfch_instance_desc d{};
  int nx = 0, ny = 0, nh = 0, rows = 0;
  int64_t npts = 0;
  RowK rk;
  ColK ck;
  dim3 row_grid, row_block, col_grid, col_block;
  size_t row_lds = 0, col_lds = 0;
  InstDev h{};            // host mirror of the device descriptor
  InstDev* dev = nullptr; // device descriptor
  double* U[2] = {nullptr, nullptr};
  int ucur = 0;
  bool has_prev = false;
  double t = 0.0, dt_prev = 0.0;
  int step_index = 0;
  int last_iters = 0;
  double* mass_part = nullptr;  // [ACC_BLOCKS]
  double* mass_out = nullptr;   // device scalar
  std::vector<void*> allocs;
};

}  // namespace

struct pfch_ctx {
  hipStream_t stream = nullptr;
  std::vector<Instance> inst;
  InstDev** d_ptrs = nullptr;
  StopRec* d_recs = nullptr;
  StopRec* h_recs = nullptr;   // pinned
  double* h_mass = nullptr;    // pinned [n]
  std::map<int, c2*> twiddles;
  std::map<int, hipGraphExec_t> graphs;       // key: chunk length K
  std::vector<hipGraph_t> graph_defs;
  int stats_detail = 1;
  std::vector<void*> allocs;
};

namespace {

int dalloc(std::vector<void*>& list, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return PFCH_E_NOMEM;
  }
  list.push_back(*p);
  return PFCH_OK;
}

int get_twiddles(pfch_ctx* ctx, int n, c2** out) {
  auto it = ctx->twiddles.find(n);
  if (it != ctx->twiddles.end()) {
    *out = it->second;
    return PFCH_OK;
  }
  std::vector<c2> h(n);
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int k = 0; k < n; ++k) {
    const long double ang = -2.0L * pi * (long double)k / (long double)n;
    h[k].x = (double)cosl(ang);
    h[k].y = (double)sinl(ang);
  }
  void* p = nullptr;
  int rc = dalloc(ctx->allocs, &p, sizeof(c2) * n);
  if (rc) return rc;
  HIPCHK(hipMemcpy(p, h.data(), sizeof(c2) * n, hipMemcpyHostToDevice));
  ctx->twiddles[n] = (c2*)p;
  *out = (c2*)p;
  return PFCH_OK;
}

uint64_t bits_of(double v) {
  uint64_t b;
  std::memcpy(&b, &v, 8);
  return b;
}
double double_of(uint64_t b) {
  double v;
  std::memcpy(&v, &b, 8);
  return v;
}

// Row pairs per row block: the most (up to 256 threads) that still leave
// at least 256 blocks; at least one.
int pick_teams(int T, int pairs) {
  int teams = 1;
  while (teams * 2 * T <= 256 && pairs % (teams * 2) == 0 && pairs / (teams * 2) >= 256) teams *= 2;
  return teams;
}
// Physical columns per column block (1, 2 or 4 of a 4-wide tile): the
// widest that keeps >= 256 blocks and <= 512 threads.
int pick_cols(int T, int H) {
  int cb = 4;
  while (cb > 1 && (cb * T > 512 || H / cb < 256)) cb >>= 1;
  return cb;
}

int setup_instance(pfch_ctx* ctx, Instance& I) {
  const pfch_instance_desc& d = I.d;
  I.nx = d.n[0];
  I.ny = d.n[1];
  I.nh = I.nx / 2;
  I.rows = I.ny;
  I.npts = (int64_t)I.nx * I.ny;
  bool ok = d.model == PFCH_PFC ? row_kernels<MODEL_PFC>(I.nx, I.rk) && col_kernels<MODEL_PFC>(I.ny, I.ck)
                                : row_kernels<MODEL_FCH>(I.nx, I.rk) && col_kernels<MODEL_FCH>(I.ny, I.ck);
  if (!ok) return PFCH_E_UNSUPPORTED;
  const int pairs = I.rows / 2;
  const int teams = pick_teams(I.rk.T, pairs);
  I.row_block = dim3(I.rk.T * teams);
  I.row_grid = dim3(pairs / teams);
  I.row_lds = (size_t)teams * I.rk.lds_elems * sizeof(c2);
  const int cb = pick_cols(I.ck.T, I.nh);
  I.col_block = dim3(I.ck.T * cb);
  I.col_grid = dim3(I.nh / cb);
  I.col_lds = (size_t)cb * I.ck.lds_elems * sizeof(c2);
  if (I.row_lds > 160 * 1024 || I.col_lds > 160 * 1024) return PFCH_E_UNSUPPORTED;

  const bool fch = d.model == PFCH_FCH;
  const int nfs = fch ? 3 : 2;  // spectral fields in S
  const int nfg = fch ? 3 : 1;  // spectral fields in G
  const int64_t fstride = (int64_t)I.rows * I.nh;
  InstDev& h = I.h;
  std::memset(&h, 0, sizeof(h));
  h.nx = I.nx;
  h.ny = I.ny;
  h.nz = 1;
  h.nh = I.nh;
  h.model = fch ? MODEL_FCH : MODEL_PFC;
  h.scheme = d.scheme == PFCH_MP ? SCHEME_MP : SCHEME_BDF2;
  h.rows = I.rows;
  h.nparts = (int)I.row_grid.x;
  const double two_pi = 6.283185307179586476925286766559;
  h.kx_scale = two_pi / d.len[0];
  h.ky_scale = two_pi / d.len[1];
  h.kz_scale = 0.0;
  h.inv_p = 1.0 / (double)I.npts;
  h.eps = d.eps;
  h.eta1 = d.eta1;
  h.eta2 = d.eta2;
  h.tau = d.tau;
  h.mobility = d.mobility;
  h.inv_mobility = 1.0 / d.mobility;
  h.s = d.s;
  h.theta_l = d.theta_l;
  const double rs = std::sqrt(d.s);
  for (int i = 0; i < 8; ++i) h.lam[i] = 0.0;
  for (int i = 0; i < d.n_eta; ++i) h.lam[i] = (1.0 - d.eta[i] * rs) / (1.0 + d.eta[i] * rs);
  h.n_eta = d.n_eta;
  h.max_iter = d.max_iter;
  h.tol_bits = bits_of(d.tol);
  h.theta = d.scheme == PFCH_MP ? 0.5 : 1.0;
  h.a = 1.0;
  h.a_over_theta = 1.0;
  h.field_stride = fstride;

  const size_t rbytes = sizeof(double) * (size_t)I.npts;
  const size_t sbytes = sizeof(c2) * (size_t)fstride;
  void* p = nullptr;
  int rc;
  for (int i = 0; i < 3; ++i) {
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    h.X[i] = (double*)p;
    if (fch) {
      if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
      h.DX[i] = (double*)p;
    }
  }
  if (fch && d.scheme == PFCH_MP) {
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    h.dun = (double*)p;
  }
  for (int i = 0; i < 2; ++i) {
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    I.U[i] = (double*)p;
  }
  if ((rc = dalloc(I.allocs, &p, sbytes * nfs))) return rc;
  h.S = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sbytes * nfg))) return rc;
  h.G = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sbytes))) return rc;
  h.ghat = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(double) * 2 * h.nparts))) return rc;
  h.part = (double*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(uint64_t) * d.max_iter))) return rc;
  h.norms = (uint64_t*)p;
  if ((rc = dalloc(I.allocs, &p, 64))) return rc;
  h.iter_base = (int32_t*)p;
  h.flags = (int32_t*)p + 1;
  if ((rc = dalloc(I.allocs, &p, sizeof(double) * ACC_BLOCKS))) return rc;
  I.mass_part = (double*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(double)))) return rc;
  I.mass_out = (double*)p;
  c2* tw = nullptr;
  if ((rc = get_twiddles(ctx, I.nx, &tw))) return rc;
  h.tw_x = tw;
  if ((rc = get_twiddles(ctx, I.ny, &tw))) return rc;
  h.tw_y = tw;
  h.tw_z = nullptr;
  if ((rc = dalloc(I.allocs, &p, sizeof(InstDev)))) return rc;
  I.dev = (InstDev*)p;
  // No instance iterates before its first setup: park the iteration base
  // beyond the cap so every iteration kernel exits at once.
  int32_t init[2] = {d.max_iter + 1, 0};
  HIPCHK(hipMemcpy(h.iter_base, init, sizeof(init), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(h.norms, 0, sizeof(uint64_t) * d.max_iter));
  return PFCH_OK;
}

int upload_desc(pfch_ctx* ctx, Instance& I) {
  HIPCHK(hipMemcpyAsync(I.dev, &I.h, sizeof(InstDev), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

int launch(const void* f, dim3 g, dim3 b, size_t lds, void** args, hipStream_t s) {
  HIPCHK(hipLaunchKernel(f, g, b, args, lds, s));
  return PFCH_OK;
}

// Build (once per chunk length) a graph running `K` iterations of every
// instance, then the chunk-end bookkeeping.
int get_graph(pfch_ctx* ctx, int K, hipGraphExec_t* out) {
  auto it = ctx->graphs.find(K);
  if (it != ctx->graphs.end()) {
    *out = it->second;
    return PFCH_OK;
  }
  hipGraph_t g;
  HIPCHK(hipGraphCreate(&g, 0));
  std::vector<hipGraphNode_t> tails;
  // Kernel arguments are copied into the node at creation time.
  for (auto& I : ctx->inst) {
    hipGraphNode_t prev = nullptr;
    for (int l = 0; l < K; ++l) {
      for (int half = 0; half < 2; ++half) {
        hipKernelNodeParams p{};
        InstDev* dev = I.dev;
        int lv = l;
        void* args[] = {&dev, &lv};
        p.func = const_cast<void*>(half == 0 ? I.ck.iter : I.rk.iter);
        p.gridDim = half == 0 ? I.col_grid : I.row_grid;
        p.blockDim = half == 0 ? I.col_block : I.row_block;
        p.sharedMemBytes = (unsigned)(half == 0 ? I.col_lds : I.row_lds);
        p.kernelParams = args;
        p.extra = nullptr;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &p));
        prev = node;
      }
    }
    tails.push_back(prev);
  }
  {
    hipKernelNodeParams p{};
    InstDev** ptrs = ctx->d_ptrs;
    int n = (int)ctx->inst.size();
    int k = K;
    void* args[] = {&ptrs, &n, &k};
    p.func = (void*)&k_chunk_end;
    p.gridDim = dim3((n + 63) / 64);
    p.blockDim = dim3(64);
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    hipGraphNode_t node;
    HIPCHK(hipGraphAddKernelNode(&node, g, tails.data(), tails.size(), &p));
  }
  hipGraphExec_t ex;
  HIPCHK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
  ctx->graph_defs.push_back(g);
  ctx->graphs[K] = ex;
  *out = ex;
  return PFCH_OK;
}

// Iterations per graph launch.  Every launch ends with one host
// synchronisation, and iterations past the stop still cost their (empty)
// launches, so the first chunk covers the predicted count exactly and
// further chunks are short.  Lengths are rounded to a small set so few
// graphs get built.
int chunk_len(int want) {
  static const int lens[] = {1, 2, 3, 4, 5, 6, 8, 10, 12, 14, 16, 20, 24, 28, 32, 40, 48, 64};
  for (int k : lens)
    if (k >= want) return k;
  return 64;
}

struct StepSetup {
  const double* un;
  const double* unm1;
  const double* xin;
  double a, b, c, theta, rho;
};

// Coefficients (eq. obj:BDF2 with backward Euler first, eq. obj:MP) and
// extrapolation factor for the next step of size dt.
StepSetup step_setup_for(const Instance& I, double dt) {
  StepSetup ss{};
  ss.un = I.U[I.ucur];
  ss.unm1 = I.has_prev ? I.U[1 - I.ucur] : I.U[I.ucur];
  ss.xin = nullptr;
  if (I.d.scheme == PFCH_MP) {
    ss.a = 1.0 / dt;
    ss.b = -1.0 / dt;
    ss.c = 0.0;
    ss.theta = 0.5;
  } else if (!I.has_prev) {
    ss.a = 1.0 / dt;
    ss.b = -1.0 / dt;
    ss.c = 0.0;
    ss.theta = 1.0;
  } else {
    const double dp = I.dt_prev;
    ss.a = 1.0 / dt + 1.0 / (dt + dp);
    ss.b = -1.0 / dt - 1.0 / dp;
    ss.c = 1.0 / dp - 1.0 / (dt + dp);
    ss.theta = 1.0;
  }
  ss.rho = I.has_prev ? dt / I.dt_prev : 0.0;
  return ss;
}

int launch_setup(pfch_ctx* ctx, Instance& I, const StepSetup& ss) {
  StepArgs sa;
  sa.un = ss.un;
  sa.unm1 = ss.unm1 ? ss.unm1 : ss.un;
  sa.xin = ss.xin;
  sa.rho = ss.rho;
  sa.a = ss.a;
  sa.theta = ss.theta;
  sa.gu = ss.b - ss.a * (1.0 - ss.theta) / ss.theta;
  sa.gm = ss.c;
  InstDev* dev = I.dev;
  int rc;
  {
    void* args[] = {&dev, &sa};
    if ((rc = launch(I.rk.setup, I.row_grid, I.row_block, I.row_lds, args, ctx->stream))) return rc;
  }
  {
    void* args[] = {&dev};
    if ((rc = launch(I.ck.setup, I.col_grid, I.col_block, I.col_lds, args, ctx->stream))) return rc;
  }
  if (I.d.model == PFCH_FCH) {
    void* args[] = {&dev};
    if ((rc = launch(I.rk.start_fch, I.row_grid, I.row_block, I.row_lds, args, ctx->stream))) return rc;
  }
  return PFCH_OK;
}

// Replay iteration chunks until every instance in `active` has stopped.
int run_iterations(pfch_ctx* ctx, const std::vector<int>& active) {
  int predicted = 1;
  for (int i : active) predicted = std::max(predicted, ctx->inst[i].last_iters);
  int K = chunk_len(ctx->inst[active[0]].last_iters > 0 ? predicted : 16);
  const int n = (int)ctx->inst.size();
  for (;;) {
    hipGraphExec_t ex;
    int rc = get_graph(ctx, K, &ex);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(ex, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->h_recs, ctx->d_recs, sizeof(StopRec) * n, hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    bool all = true;
    for (int i : active) {
      const StopRec& r = ctx->h_recs[i];
      if (r.stop_iter < 0 && !(r.flags & FLAG_PRECOND)) all = false;
    }
    if (all) return PFCH_OK;
    K = chunk_len(2);
  }
}

int status_of(const Instance& I, const StopRec& r, int* iters, double* dnorm) {
  const double nv = double_of(r.norm_bits);
  *dnorm = nv;
  if (r.flags & FLAG_PRECOND) {
    *iters = 0;
    return PFCH_E_PRECOND;
  }
  if (r.stop_iter >= I.d.max_iter) {
    *iters = I.d.max_iter;
    return PFCH_E_NOCONV;
  }
  *iters = r.stop_iter + 1;
  if (!std::isfinite(nv)) return PFCH_E_NONFINITE;
  return PFCH_OK;
}

int betas_host(pfch_ctx* ctx, Instance& I, double a, double out[4]) {
  std::vector<double> part(2 * I.h.nparts);
  HIPCHK(hipMemcpyAsync(part.data(), I.h.part, sizeof(double) * part.size(), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  double s0 = 0.0, s1 = 0.0;
  for (int i = 0; i < I.h.nparts; ++i) {
    s0 += part[2 * i];
    s1 += part[2 * i + 1];
  }
  out[0] = a / I.d.mobility;
  if (I.d.model == PFCH_PFC) {
    out[1] = std::fabs(s0 * I.h.inv_p);
    out[2] = -2.0;
    out[3] = 1.0;
  } else {
    const double e2 = I.d.eps * I.d.eps;
    out[1] = std::fabs(s0 * I.h.inv_p);
    out[2] = std::fabs(s1 * I.h.inv_p);
    out[3] = e2 * e2;
  }
  return PFCH_OK;
}

int fft_pairs_of(const Instance& I, int iters) {
  // real-field transform pairs: iterations use (nfwd + ninv)/2, setup adds
  // the transforms of g, x0 (FCH) and u^n (FCH midpoint).
  const bool fch = I.d.model == PFCH_FCH;
  const int per_iter = fch ? 5 : 3;  // forward + inverse real fields
  const int setup = fch ? (I.d.scheme == PFCH_MP ? 2 * 3 + 3 : 2 * 2 + 3) : 1 + 2;
  return (per_iter * iters + setup + 1) / 2;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

int pfch_version(void) { return PFCH_VERSION; }

const char* pfch_strerror(int code) {
  switch (code) {
    case PFCH_OK: return "ok";
    case PFCH_E_INVAL: return "invalid argument";
    case PFCH_E_NOMEM: return "out of memory";
    case PFCH_E_HIP: return "HIP runtime error";
    case PFCH_E_NOCONV: return "PAGD did not reach the tolerance within max_iter";
    case PFCH_E_NONFINITE: return "non-finite value in the PAGD iteration";
    case PFCH_E_PRECOND: return "averaged-Newton preconditioner not positive";
    case PFCH_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown error";
  }
}

int pfch_validate_desc(const pfch_instance_desc* d) {
  if (!d) return PFCH_E_INVAL;
  if (d->model != PFCH_PFC && d->model != PFCH_FCH) return PFCH_E_INVAL;
  if (d->scheme != PFCH_BDF2 && d->scheme != PFCH_MP) return PFCH_E_INVAL;
  if (d->reserved != 0) return PFCH_E_INVAL;
  if (d->ndim != 2 && d->ndim != 3) return PFCH_E_INVAL;
  for (int a = 0; a < d->ndim; ++a) {
    if (d->n[a] < 2 || !(d->len[a] > 0.0) || !std::isfinite(d->len[a])) return PFCH_E_INVAL;
  }
  if (!std::isfinite(d->eps) || !std::isfinite(d->eta1) || !std::isfinite(d->eta2) ||
      !std::isfinite(d->tau))
    return PFCH_E_INVAL;
  if (d->model == PFCH_FCH && !(d->eps > 0.0)) return PFCH_E_INVAL;
  if (!(d->mobility > 0.0) || !std::isfinite(d->mobility)) return PFCH_E_INVAL;
  if (!(d->s > 0.0) || !std::isfinite(d->s)) return PFCH_E_INVAL;
  if (!(d->tol > 0.0) || !std::isfinite(d->tol)) return PFCH_E_INVAL;
  if (!(d->theta_l > 0.0) || !std::isfinite(d->theta_l)) return PFCH_E_INVAL;
  if (d->n_eta < 1 || d->n_eta > 8) return PFCH_E_INVAL;
  for (int i = 0; i < d->n_eta; ++i)
    if (!(d->eta[i] >= 0.0) || !std::isfinite(d->eta[i])) return PFCH_E_INVAL;
  if (d->max_iter < 1 || d->max_iter > 1000000) return PFCH_E_INVAL;
  if (d->guess != 0) return PFCH_E_UNSUPPORTED;
  if (d->ndim != 2) return PFCH_E_UNSUPPORTED;
  if (!supported_len(d->n[0]) || !supported_len(d->n[1])) return PFCH_E_UNSUPPORTED;
  return PFCH_OK;
}

void pfch_destroy(pfch_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : ctx->graph_defs) (void)hipGraphDestroy(g);
  for (auto& I : ctx->inst)
    for (void* p : I.allocs) (void)hipFree(p);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->h_recs) (void)hipHostFree(ctx->h_recs);
  if (ctx->h_mass) (void)hipHostFree(ctx->h_mass);
  delete ctx;
}

int pfch_create(const pfch_instance_desc* descs, int32_t n_inst, void* hip_stream, pfch_ctx** out) {
  if (!out || !descs || n_inst < 1) return PFCH_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < n_inst; ++i) {
    int rc = pfch_validate_desc(&descs[i]);
    if (rc) return rc;
  }
  auto ctx = new (std::nothrow) pfch_ctx();
  if (!ctx) return PFCH_E_NOMEM;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->inst.resize(n_inst);
  int rc = PFCH_OK;
  void* p = nullptr;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(StopRec) * n_inst))) goto fail;
  ctx->d_recs = (StopRec*)p;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(InstDev*) * n_inst))) goto fail;
  ctx->d_ptrs = (InstDev**)p;
  if (hipHostMalloc((void**)&ctx->h_recs, sizeof(StopRec) * n_inst, 0) != hipSuccess) {
    rc = PFCH_E_NOMEM;
    goto fail;
  }
  if (hipHostMalloc((void**)&ctx->h_mass, sizeof(double) * n_inst, 0) != hipSuccess) {
    rc = PFCH_E_NOMEM;
    goto fail;
  }
  {
    std::vector<InstDev*> ptrs(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      Instance& I = ctx->inst[i];
      I.d = descs[i];
      if ((rc = setup_instance(ctx, I))) goto fail;
      I.h.rec = ctx->d_recs + i;
      if ((rc = upload_desc(ctx, I))) goto fail;
      ptrs[i] = I.dev;
    }
    if (hipMemcpy(ctx->d_ptrs, ptrs.data(), sizeof(InstDev*) * n_inst, hipMemcpyHostToDevice) !=
        hipSuccess) {
      rc = PFCH_E_HIP;
      goto fail;
    }
    std::vector<StopRec> recs(n_inst);
    for (auto& r : recs) {
      r.stop_iter = 0;
      r.flags = 0;
      r.norm_bits = 0;
    }
    if (hipMemcpy(ctx->d_recs, recs.data(), sizeof(StopRec) * n_inst, hipMemcpyHostToDevice) !=
        hipSuccess) {
      rc = PFCH_E_HIP;
      goto fail;
    }
    // Kernels that need more than the default dynamic LDS.
    for (auto& I : ctx->inst) {
      const void* fs[] = {I.rk.iter, I.rk.setup, I.rk.start_fch};
      for (const void* f : fs)
        if (f && I.row_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)I.row_lds);
      const void* gs[] = {I.ck.iter, I.ck.setup};
      for (const void* f : gs)
        if (f && I.col_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)I.col_lds);
    }
  }
  *out = ctx;
  return PFCH_OK;
fail:
  pfch_destroy(ctx);
  return rc;
}

int pfch_set_stats_detail(pfch_ctx* ctx, int32_t detail) {
  if (!ctx || detail < 0 || detail > 1) return PFCH_E_INVAL;
  ctx->stats_detail = detail;
  return PFCH_OK;
}

int pfch_time_kernels(pfch_ctx* ctx, double dt, int32_t reps, double out[2]) {
  if (!ctx || !out || reps < 1 || !(dt > 0.0) || !std::isfinite(dt)) return PFCH_E_INVAL;
  Instance& I = ctx->inst[0];
  int rc;
  if ((rc = launch_setup(ctx, I, step_setup_for(I, dt)))) return rc;
  hipEvent_t e[3];
  for (auto& ev : e) HIPCHK(hipEventCreate(&ev));
  InstDev* dev = I.dev;
  int l0 = 0;  // iteration 0 after setup: every launch does full work
  void* args[] = {&dev, &l0};
  HIPCHK(hipEventRecord(e[0], ctx->stream));
  for (int r = 0; r < reps; ++r)
    if ((rc = launch(I.ck.iter, I.col_grid, I.col_block, I.col_lds, args, ctx->stream))) return rc;
  HIPCHK(hipEventRecord(e[1], ctx->stream));
  for (int r = 0; r < reps; ++r)
    if ((rc = launch(I.rk.iter, I.row_grid, I.row_block, I.row_lds, args, ctx->stream))) return rc;
  HIPCHK(hipEventRecord(e[2], ctx->stream));
  HIPCHK(hipEventSynchronize(e[2]));
  float t0 = 0.f, t1 = 0.f;
  HIPCHK(hipEventElapsedTime(&t0, e[0], e[1]));
  HIPCHK(hipEventElapsedTime(&t1, e[1], e[2]));
  for (auto& ev : e) (void)hipEventDestroy(ev);
  out[0] = 1e3 * t0 / reps;
  out[1] = 1e3 * t1 / reps;
  // park the instance so later chunk launches leave it alone
  int32_t park = I.d.max_iter + 1;
  HIPCHK(hipMemcpyAsync(I.h.iter_base, &park, sizeof(park), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

int pfch_get_launch_config(pfch_ctx* ctx, int32_t inst, int64_t out[6]) {
  if (!ctx || !out || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  const Instance& I = ctx->inst[inst];
  out[0] = I.row_grid.x;
  out[1] = I.row_block.x;
  out[2] = (int64_t)I.row_lds;
  out[3] = I.col_grid.x;
  out[4] = I.col_block.x;
  out[5] = (int64_t)I.col_lds;
  return PFCH_OK;
}

int pfch_set_state(pfch_ctx* ctx, int32_t inst, const double* u_n, const double* u_nm1, double t,
                   double dt_prev, int32_t step_index) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !u_n) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  if (u_nm1 && !(dt_prev > 0.0)) return PFCH_E_INVAL;
  const size_t bytes = sizeof(double) * (size_t)I.npts;
  HIPCHK(hipMemcpyAsync(I.U[I.ucur], u_n, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (u_nm1) HIPCHK(hipMemcpyAsync(I.U[1 - I.ucur], u_nm1, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  I.has_prev = u_nm1 != nullptr;
  I.t = t;
  I.dt_prev = u_nm1 ? dt_prev : 0.0;
  I.step_index = step_index;
  return PFCH_OK;
}

int pfch_get_state(pfch_ctx* ctx, int32_t inst, double* u_n, double* u_nm1, double* t, double* dt_prev,
                   int32_t* step_index) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  const size_t bytes = sizeof(double) * (size_t)I.npts;
  if (u_n) HIPCHK(hipMemcpyAsync(u_n, I.U[I.ucur], bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (u_nm1 && I.has_prev)
    HIPCHK(hipMemcpyAsync(u_nm1, I.U[1 - I.ucur], bytes, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (t) *t = I.t;
  if (dt_prev) *dt_prev = I.dt_prev;
  if (step_index) *step_index = I.step_index;
  return PFCH_OK;
}

int pfch_step(pfch_ctx* ctx, const double* dt, pfch_stats* st) {
  if (!ctx || !dt) return PFCH_E_INVAL;
  const int n = (int)ctx->inst.size();
  for (int i = 0; i < n; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return PFCH_E_INVAL;
  std::vector<int> active(n);
  std::vector<double> as(n);
  int rc;
  for (int i = 0; i < n; ++i) {
    Instance& I = ctx->inst[i];
    active[i] = i;
    const StepSetup ss = step_setup_for(I, dt[i]);
    as[i] = ss.a;
    if ((rc = launch_setup(ctx, I, ss))) return rc;
  }
  if ((rc = run_iterations(ctx, active))) return rc;
  int first_err = PFCH_OK;
  std::vector<int> status(n), iters(n);
  std::vector<double> dn(n);
  const bool want_mass = st && ctx->stats_detail > 0;
  for (int i = 0; i < n; ++i) {
    Instance& I = ctx->inst[i];
    status[i] = status_of(I, ctx->h_recs[i], &iters[i], &dn[i]);
    if (status[i] != PFCH_OK) {
      if (first_err == PFCH_OK) first_err = status[i];
      continue;
    }
    const int slot = (ctx->h_recs[i].stop_iter + 1) % 3;
    double* dst = I.U[1 - I.ucur];
    int64_t np = I.npts;
    double* part = want_mass ? I.mass_part : nullptr;
    const double* src = I.h.X[slot];
    void* args[] = {&src, &dst, &np, &part};
    if ((rc = launch((const void*)&k_copy_sum, dim3(ACC_BLOCKS), dim3(ACC_THREADS), 0, args, ctx->stream)))
      return rc;
    if (want_mass) {
      int nb = ACC_BLOCKS;
      double scale = 1.0 / (double)I.npts;
      double* o = I.mass_out;
      void* a2[] = {&I.mass_part, &nb, &scale, &o};
      if ((rc = launch((const void*)&k_sum_parts, dim3(1), dim3(1), 0, a2, ctx->stream))) return rc;
      HIPCHK(hipMemcpyAsync(&ctx->h_mass[i], I.mass_out, sizeof(double), hipMemcpyDeviceToHost,
                            ctx->stream));
    }
    I.ucur = 1 - I.ucur;
    I.has_prev = true;
    I.dt_prev = dt[i];
    I.t += dt[i];
    I.step_index += 1;
    I.last_iters = iters[i];
  }
  if (st) {
    if (want_mass) HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i) {
      Instance& I = ctx->inst[i];
      pfch_stats& s = st[i];
      std::memset(&s, 0, sizeof(s));
      s.status = status[i];
      s.iters = iters[i];
      s.dnorm_inf = dn[i];
      s.fft_pairs = fft_pairs_of(I, iters[i]);
      s.mass = (want_mass && status[i] == PFCH_OK) ? ctx->h_mass[i] : NAN;
      if (ctx->stats_detail > 0) {
        if ((rc = betas_host(ctx, I, as[i], s.beta))) return rc;
      } else {
        for (double& b : s.beta) b = NAN;
      }
    }
  }
  return first_err;
}

int pfch_solve(pfch_ctx* ctx, int32_t inst, double a, double b, double c, const double* u_n,
               const double* u_nm1, double* x, pfch_stats* st) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !u_n || !x) return PFCH_E_INVAL;
  if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c)) return PFCH_E_INVAL;
  if (c != 0.0 && !u_nm1) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  StepSetup ss{};
  ss.un = u_n;
  ss.unm1 = u_nm1 ? u_nm1 : u_n;
  ss.xin = x;
  ss.a = a;
  ss.b = b;
  ss.c = c;
  ss.theta = I.d.scheme == PFCH_MP ? 0.5 : 1.0;
  ss.rho = 0.0;
  int rc;
  if ((rc = launch_setup(ctx, I, ss))) return rc;
  std::vector<int> active{inst};
  if ((rc = run_iterations(ctx, active))) return rc;
  int iters = 0;
  double dn = 0.0;
  const int status = status_of(I, ctx->h_recs[inst], &iters, &dn);
  if (status == PFCH_OK || status == PFCH_E_NOCONV || status == PFCH_E_NONFINITE) {
    const StopRec& r = ctx->h_recs[inst];
    const int last = status == PFCH_E_NOCONV ? I.d.max_iter : r.stop_iter + 1;
    const size_t bytes = sizeof(double) * (size_t)I.npts;
    HIPCHK(hipMemcpyAsync(x, I.h.X[last % 3], bytes, hipMemcpyDeviceToDevice, ctx->stream));
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  I.last_iters = iters;
  if (st) {
    std::memset(st, 0, sizeof(*st));
    st->status = status;
    st->iters = iters;
    st->dnorm_inf = dn;
    st->fft_pairs = fft_pairs_of(I, iters);
    st->mass = NAN;
    if ((rc = betas_host(ctx, I, a, st->beta))) return rc;
  }
  return status;
}

}  // extern "C"
