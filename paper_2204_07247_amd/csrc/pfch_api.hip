// Host runtime of libpfch: context, workspaces, grouped launches, iteration
// graphs and the C ABI.
//
// Instances that share (model, Nx, Ny) form a group; every kernel launch
// covers a whole group (block b works on member b / bpi).  One iteration
// graph holds, per group, a chain of column/row kernels for K iterations;
// the chains of different groups are independent and may run concurrently.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "../../include/pfch.h"
#include "kernels2d.hpp"
#include "plans.hpp"
#include "fno.hpp"

using namespace pfch;

namespace {

// Implicit-midpoint family (u_breve blends u^n) and the linear IMEX schemes.
inline bool scheme_mp(int s) { return s == PFCH_MP || s == PFCH_LMP; }
inline bool scheme_imex(int s) { return s == PFCH_LBDF2 || s == PFCH_LMP; }

// ---------------------------------------------------------------------------
// Small kernels: end of a chunk of iterations, accept, mass reduction.
// ---------------------------------------------------------------------------
// One block: every instance's stop record for the chunk just run, mirrored
// into pinned host memory, then the host-visible chunk counter.  A group of
// S lanes (a power of two up to 64, S >= K where the block allows) scans an
// instance's chunk: each lane tests one iteration's norm and a ballot picks
// the first that stops the solve, so the norms are read in parallel rather
// than one dependent load per iteration.
//
// Host-visible writes, in this order, each group separated from the next by
// a system-scope fence and a block barrier: (1) every mirror's stop_iter,
// flags and norm; (2) every mirror's chunk number; (3) the chunk counter.
// The host waits for (3) and then uses a mirror only if its chunk number
// (2) is the chunk it waited for, so a record from an earlier chunk is never
// taken for this chunk's.
__device__ __forceinline__ int chunk_group_size(int K, int n) {
  int S = 1;
  while (S < K && S < 64) S *= 2;
  while (S > 1 && (long long)S * n > 1024) S /= 2;
  return S;
}

__global__ __launch_bounds__(1024) void k_chunk_end(InstDev* const* insts, int n, int K,
                                                    uint32_t* __restrict__ seq_dev,
                                                    uint32_t* __restrict__ seq_host) {
  const int S = chunk_group_size(K, n);
  const int g = threadIdx.x / S, r = threadIdx.x % S, ngroups = blockDim.x / S;
  const int wl = threadIdx.x & 63, gbase = wl - r;  // group's first lane in the wave
  const uint32_t tag = *seq_dev + 1;  // this chunk's number (seq_dev changes only below)
  const uint64_t gmask = S == 64 ? ~0ull : ((1ull << S) - 1) << gbase;
  for (int i = g; i < n; i += ngroups) {
    InstDev* I = insts[i];
    StopRec* rec = I->rec;
    const int base = *I->iter_base;
    const int before = rec->stop_iter;
    const int maxit = I->max_iter;
    int stop = -1;
    uint64_t nb = 0;
    if (before < 0 && base < maxit + 1) {
      for (int j0 = base; j0 < base + K && stop < 0; j0 += S) {
        const int jj = j0 + r;
        bool hit = false;
        uint64_t b = 0;
        if (jj < base + K) {
          if (jj >= maxit) {
            hit = true;  // the cap: stop at max_iter with the last norm
            b = I->norms[maxit - 1];
          } else {
            b = I->norms[jj];
            hit = b < I->tol_bits || b >= INF_BITS;
          }
        }
        const uint64_t m = (uint64_t)__ballot(hit) & gmask;
        if (m) {
          const int f = __ffsll((long long)m) - 1;  // lane in the wave
          stop = min(j0 + (f - gbase), maxit);
          nb = __shfl(b, f);
        }
      }
    }
    if (r == 0) {
      if (stop >= 0) {
        rec->stop_iter = stop;
        rec->norm_bits = nb;
      }
      rec->flags |= *I->flags;
      const bool stopped = rec->stop_iter >= 0 || (rec->flags & FLAG_PRECOND);
      *I->iter_base = stopped ? maxit + 1 : base + K;
      // the accept that follows in the graph copies a solution once, in the
      // chunk that ended its solve
      const bool ended = before < 0 && rec->stop_iter >= 0;
      I->acc_now = ended ? I->acc_dst : nullptr;
      I->acc_lnow = ended ? I->acc_ldst : nullptr;
      StopRec* h = I->rec_host;  // the host polls this copy
      h->stop_iter = rec->stop_iter;
      h->flags = rec->flags;
      h->norm_bits = rec->norm_bits;
    }
  }
  __threadfence_system();
  __syncthreads();
  if (r == 0)
    for (int i = g; i < n; i += ngroups) insts[i]->rec_host->seq = tag;
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0) {
    *seq_dev = tag;
    *seq_host = tag;
    __threadfence_system();
  }
}

// Park instances: no iteration kernel works on them and no in-graph accept
// copies for them until their next set-up.  Used when a queued set-up is
// discarded and after a residual evaluation.  One thread per instance.
__global__ __launch_bounds__(256) void k_park(InstDev* const* insts, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  InstDev* I = insts[i];
  *I->iter_base = I->max_iter + 1;
  I->acc_dst = nullptr;
  I->acc_ldst = nullptr;
  I->acc_now = nullptr;
  I->acc_lnow = nullptr;
}

// Threads of the chunk-end block: one group of S lanes per instance (up to
// 1024 threads; more instances loop), whole waves.
inline int chunk_end_threads(int K, int n) {
  int S = 1;
  while (S < K && S < 64) S *= 2;
  while (S > 1 && (long long)S * n > 1024) S /= 2;
  const long long t = std::min<long long>(1024, (long long)S * n);
  return (int)((t + 63) / 64 * 64);
}

constexpr int ACC_BLOCKS = 1024, ACC_THREADS = 256;

// Accept: copy every converged instance's solution x_{stop+1} to its new
// u^n slot (dsts[i]; null = not accepted) and, if part is given, write
// gridDim.x partial sums of it per instance (fixed order).
// Up to ACC_INLINE destinations travel by value with the launch.
constexpr int ACC_INLINE = 16;
struct AccDsts {
  double* p[ACC_INLINE];
};
// check >= 1: accept only an instance whose solve has ended well (the test
// the host applies to the same record), so the accept can run behind the
// iterations before the host has seen the outcome; accepting the same
// solution twice writes the same values.  check = 2 (inside the chunk
// graph): the destination is the one the step set-up published, in the chunk
// that ended the solve only (null otherwise, and for solves that are not
// accepted this way).
__global__ __launch_bounds__(ACC_THREADS) void k_accept(InstDev* const* __restrict__ insts,
                                                        double* const* __restrict__ dsts,
                                                        double* __restrict__ part, AccDsts inl, int check) {
  __shared__ double red[ACC_THREADS / 64];
  const int i = blockIdx.y;
  double* dst = check == 2 ? insts[i]->acc_now : dsts ? dsts[i] : inl.p[i];
  if (!dst) return;
  const InstDev* I = insts[i];
  if (check) {  // the same test as status_of on the host
    const StopRec r = *I->rec;
    if ((r.flags & FLAG_PRECOND) || r.stop_iter < 0 || r.stop_iter >= I->max_iter || r.norm_bits >= INF_BITS)
      return;
  }
  const int slot = (I->rec->stop_iter + 1) % 3;
  const GLB double* src = gp((const double*)I->X[slot]);
  GLB double* d = gp(dst);
  const int64_t n = (int64_t)I->nx * I->ny * I->nz;
  double s = 0.0;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (int64_t)gridDim.x * blockDim.x) {
    const double v = src[k];
    d[k] = v;
    s += v;
  }
  if (check == 2 && I->acc_lnow) {  // FCH: keep the solution's Laplacian too
    const GLB double* ls = gp((const double*)I->DX[slot]);
    GLB double* ld = gp(I->acc_lnow);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (int64_t)gridDim.x * blockDim.x)
      ld[k] = ls[k];
  }
  const double b = block_sum(s, red);
  if (threadIdx.x == 0 && part) part[(int64_t)i * gridDim.x + blockIdx.x] = b;
}

// One block per instance: its nb partial sums in a fixed order (strided per
// thread, then the block's fixed reduction tree).
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nb, int n,
                                                   const double* scale, double* out) {
  __shared__ double red[4];
  const int i = blockIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x) s += part[(int64_t)i * nb + k];
  const double b = block_sum(s, red);
  if (threadIdx.x == 0) {
    out[i] = b * scale[i];
    __threadfence_system();  // out may be pinned host memory
  }
}

// ---------------------------------------------------------------------------
// Static scratch of the allocation-free R(v) entry point (pfch_rhs_noalloc):
// the source and destination pointers in the first 256 bytes, then up to
// three tiled spectral fields.  Each device holds its own copy until the
// process ends; host code uses only the per-device address that
// hipGetSymbolAddress returns (scratch_for_device), never the array's name.
// ---------------------------------------------------------------------------
constexpr size_t SCRATCH_SPECTRAL_BYTES = (size_t)32 << 20;
constexpr size_t SCRATCH_PTR_BYTES = 256;
static __device__ __align__(256) unsigned char scratch[SCRATCH_PTR_BYTES + SCRATCH_SPECTRAL_BYTES];

__global__ __launch_bounds__(64) void k_rhs_ptrs(const double** slot, const double* src, double* dst) {
  if (threadIdx.x == 0) {
    slot[0] = src;
    slot[1] = dst;
  }
}

// ---------------------------------------------------------------------------
// Host structures.
// ---------------------------------------------------------------------------
#define HIPCHK(x)                            \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return PFCH_E_HIP; \
  } while (0)

struct Instance {
  pfch_instance_desc d{};
  int nx = 0, ny = 0, nz = 1, nh = 0, rows = 0;
  int64_t npts = 0;
  int group = -1;
  InstDev h{};             // host mirror of the device descriptor
  InstDev* dev = nullptr;  // device descriptor
  InstDev** d_solo = nullptr;  // device array {dev}: single-instance launches
  double* U[2] = {nullptr, nullptr};
  double* dU[2] = {nullptr, nullptr};  // FCH: Laplacians of U, kept by pfch_step's accept
  int lap_levels = 0;                  // how many of dU match the history
  int ucur = 0;
  bool has_prev = false;
  double t = 0.0, dt_prev = 0.0;
  int step_index = 0;
  int last_iters = 0;
  pfch_fno* fno = nullptr;  // learned initial guess (not owned)
  Resampler* fno_rs = nullptr;  // its resampler when the network's grid is coarser (owned by the network)
  double fno_norm[4] = {0, 1, 1, 1};
  double* xguess = nullptr;  // learned guess buffer (allocated on first attach)
  double* gpart = nullptr;   // GUESS_BLOCKS partial sums of the network output, then its mean
  // gain of the learned correction: gbuf[0..1] the gain (read one, written
  // the other, gain_par the one to read), then 2 GUESS_BLOCKS partials;
  // gcor the last guess's correction; gain_ready: the last step took its
  // learned guess and was accepted, so the next guess can update the gain
  double* gbuf = nullptr;
  float* gcor = nullptr;
  int gain_par = 0;
  bool gain_ready = false;
  bool gain_fresh = false;  // the last learned guess's gain came from its previous step's partials
  // gate of the learned guess: while off, steps take the extrapolated guess
  // (no network call) and lg_wait counts the steps to the next probe
  bool lg_off = false;
  int lg_wait = 0;
  int lg_probe = 0;  // learned steps left in a probe of the network
  int lg_fails = 0;  // probes in a row that closed the gate again
  // adaptive stepping (buffers allocated on first use)
  double* Um2 = nullptr;     // u^{n-2}
  double* R[3] = {nullptr, nullptr, nullptr};  // R(u^n), R(u^{n-1}), R(u~)
  int hist = 1;              // solutions held: u^n, u^{n-1}, u^{n-2}
  bool r_valid = false;      // R[0] (and R[1] when hist >= 2) match the history
  double dt_nm1 = 0.0;       // dt_{n-1}, valid when hist == 3
  double* uprobe = nullptr;  // statistics detail 2: u^{n-1} of the step being taken
  std::vector<void*> allocs;
};

struct Group {
  int model = 0, scheme = 0, nx = 0, ny = 0;
  // iteration kernels and their launch geometry (autotuned)
  RowK rk;
  ColK ck;
  dim3 row_block, col_block;
  int row_bpi = 0, col_bpi = 0;  // blocks per instance
  size_t row_lds = 0, col_lds = 0;
  // step-setup kernels: always the default plan and geometry, so that the
  // partial sums of the averaged-Newton constants do not depend on tuning
  RowK rs;
  ColK cs;
  dim3 srow_block, scol_block;
  int srow_bpi = 0, scol_bpi = 0;
  size_t srow_lds = 0, scol_lds = 0;
  std::vector<RowK> ralts;  // alternative iteration plans
  std::vector<ColK> calts;
  // 3D (PFC): y- and z-pass kernels and geometry
  int ndim = 2, nz = 1, rows = 0;
  Y3K y3, y3d;  // current and default plan
  Z3K z3, z3d;
  std::vector<Y3K> y3alts;
  std::vector<Z3K> z3alts;
  dim3 y3_block, z3_block;
  int y3_bpi = 0, z3_bpi = 0;
  size_t y3_lds = 0, z3_lds = 0;
  std::vector<int> members;
  InstDev** d_members = nullptr;
  StepArgs* d_args = nullptr;
  StepArgs* h_args = nullptr;  // pinned
  const double** d_rptr = nullptr;  // R(v) launches: [member] sources, then destinations
  const double** h_rptr = nullptr;  // pinned staging
};

}  // namespace

struct pfch_fno {
  Fno f;
};

struct pfch_ctx {
  hipStream_t stream = nullptr;
  // Set-up of the next step enqueued at the end of pfch_step (same dt as
  // the last two calls): the next pfch_step with that dt skips it.  Every
  // other call that touches instance state or workspaces drops it.
  bool spec = false;
  std::vector<double> last_dt;  // step sizes of the last pfch_step
  std::vector<int> spec_guess;
  std::vector<double> spec_a;
  std::vector<Instance> inst;
  std::vector<Group> groups;
  InstDev** d_ptrs = nullptr;  // all instances
  StopRec* d_recs = nullptr;
  StopRec* h_recs = nullptr;   // pinned; written by the chunk-end kernel
  std::vector<StopRec> recs;   // the records of the last chunk, copied once its number checked
  int32_t* h_scratch = nullptr;  // pinned staging for small uploads
  uint32_t* d_seq = nullptr;     // chunk counter (device) and its pinned mirror
  uint32_t* h_seq = nullptr;
  uint32_t seq = 0;              // chunks launched
  int acc_blocks = 1;            // accept blocks per instance (<= ACC_BLOCKS)
  double** d_dsts = nullptr;   // accept destinations
  double** h_dsts = nullptr;   // pinned
  double* d_part = nullptr;    // [n][ACC_BLOCKS]
  double* d_scale = nullptr;   // 1/P per instance
  double* d_mass = nullptr;    // device address of h_mass
  double* h_mass = nullptr;    // pinned, coherent
  double* d_gain = nullptr;    // device address of h_gain
  double* h_gain = nullptr;    // pinned, coherent: gain of each instance's last learned guess
  EstArgs* d_est = nullptr;    // adaptive error estimate, per instance
  EstArgs* h_est = nullptr;    // pinned
  double* d_est_part = nullptr;  // [n][2][EST_BLOCKS]
  double* h_est_part = nullptr;  // pinned
  std::map<int, c2*> twiddles;
  std::map<int, hipGraphExec_t> graphs;  // key: chunk length K
  std::vector<hipGraph_t> graph_defs;
  int stats_detail = 1;
  int device = -1;             // device current at pfch_create
  void* scratch = nullptr;     // that device's address of the static scratch
  std::vector<void*> allocs;
  std::vector<void*> host_allocs;
};

namespace {

// With PFCH_DEBUG set in the environment, failed allocations are reported
// on stderr with the runtime's error string.
void alloc_failed(const char* what, size_t bytes, hipError_t e) {
  const char* dbg = std::getenv("PFCH_DEBUG");
  if (dbg && dbg[0] && dbg[0] != '0')
    std::fprintf(stderr, "pfch: %s of %zu bytes failed: %s\n", what, bytes, hipGetErrorString(e));
}

int dalloc(std::vector<void*>& list, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  const hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    alloc_failed("hipMalloc", bytes, e);
    *p = nullptr;
    return PFCH_E_NOMEM;
  }
  list.push_back(*p);
  return PFCH_OK;
}

// Pinned host memory, zero-filled.  coherent: kernels write into it while
// the host polls it (stop records, the chunk counter), so device writes must
// reach host memory in the order their fences give, with no caching in the
// device's L2.
int halloc(std::vector<void*>& list, void** p, size_t bytes, bool coherent = false) {
  const unsigned flags = coherent ? hipHostMallocMapped | hipHostMallocCoherent : hipHostMallocDefault;
  const hipError_t e = hipHostMalloc(p, bytes, flags);
  if (e != hipSuccess) {
    alloc_failed("hipHostMalloc", bytes, e);
    *p = nullptr;
    return PFCH_E_NOMEM;
  }
  std::memset(*p, 0, bytes);
  list.push_back(*p);
  return PFCH_OK;
}

// Address of `scratch` on device `dev`, looked up once per device (with
// that device current) and kept for the process.
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex& scratch_mutex() {
  static std::mutex m;
  return m;
}
void* g_scratch_ptr[SCRATCH_MAX_DEVICES] = {};
int scratch_for_device(int dev, void** out) {
  *out = nullptr;
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return PFCH_E_UNSUPPORTED;
  std::lock_guard<std::mutex> lk(scratch_mutex());
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return PFCH_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
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

// Launch geometry depends on the grid shape only (not on how many
// instances share a launch), so an instance computes bitwise the same
// result alone or in a batch (the averaged-Newton partial sums are per
// block).
// Row pairs per row block: the most (up to 256 threads) that still leave
// at least 256 blocks per instance; at least one.
int pick_teams(int T, int pairs) {
  int teams = 1;
  while (teams * 2 * T <= 256 && pairs % (teams * 2) == 0 && pairs / (teams * 2) >= 256) teams *= 2;
  return teams;
}
// Physical columns per column block (1, 2 or 4 of a 4-wide tile): the
// widest that keeps >= 256 blocks per instance and <= 512 threads.
int pick_cols(int T, int H) {
  int cb = 4;
  while (cb > 1 && (cb * T > 512 || H / cb < 256)) cb >>= 1;
  return cb;
}

int setup_instance(pfch_ctx* ctx, Instance& I, int nparts) {
  const pfch_instance_desc& d = I.d;
  const bool fch = d.model == PFCH_FCH;
  const int nfs = fch ? 3 : 2;  // spectral fields in S
  const int nfg = fch ? 3 : 1;  // spectral fields in G
  const int64_t fstride = (int64_t)I.rows * I.nh;
  InstDev& h = I.h;
  std::memset(&h, 0, sizeof(h));
  h.nx = I.nx;
  h.ny = I.ny;
  h.nz = I.nz;
  h.nh = I.nh;
  h.model = fch ? MODEL_FCH : MODEL_PFC;
  h.scheme = scheme_mp(d.scheme) ? SCHEME_MP : SCHEME_BDF2;
  h.rows = I.rows;
  h.nparts = nparts;
  const double two_pi = 6.283185307179586476925286766559;
  h.kx_scale = two_pi / d.len[0];
  h.ky_scale = two_pi / d.len[1];
  h.kz_scale = I.nz > 1 ? two_pi / d.len[2] : 0.0;
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
  h.n_eta = d.n_eta > 0 ? d.n_eta : 1;  // n_eta = 0: lambda = 0, plain PGD (Alg. 1)
  h.max_iter = d.max_iter;
  h.tol_bits = bits_of(d.tol);
  h.theta = scheme_mp(d.scheme) ? 0.5 : 1.0;
  if (scheme_imex(d.scheme)) {
    // A linear IMEX step (eq. eqn:FCH-semidis-simplicit) is one iteration
    // of the same kernels from y = u^n + rho (u^n - u^{n-1}) (LMP: the
    // unknown's midpoint with u^n is then ((2 + rho) u^n - rho u^{n-1})/2,
    // LBDF2: y itself), with unit step, the preconditioner replaced by the
    // symbol of the implicit part, l(k) = beta0 + beta2 q + beta4 q^2 with
    // weight theta, and no tolerance: d = (a/M + theta q l)^{-1} (-residual)
    // solves the linear step exactly and u^{n+1} = y + d.
    h.imex = 1;
    h.s = 1.0;
    for (int i = 0; i < 8; ++i) h.lam[i] = 0.0;
    h.n_eta = 1;
    h.tol_bits = INF_BITS;
    h.theta_l = h.theta;
    if (fch) {
      h.imex_b0 = 1.0 - 2.0 * d.tau * d.tau + d.eta2;  // kappa0
      h.imex_b2 = 1.0;                                  // kappa2
    } else {
      h.imex_b0 = 1.0;  // (1 - q)^2 = 1 - 2 q + q^2
      h.imex_b2 = -2.0;
    }
  }
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
  if (fch && scheme_mp(d.scheme)) {
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    h.dun = (double*)p;
  }
  for (int i = 0; i < 2; ++i) {
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    I.U[i] = (double*)p;
    if (fch && I.nz == 1) {
      if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
      I.dU[i] = (double*)p;
    }
  }
  if ((rc = dalloc(I.allocs, &p, sbytes * nfs))) return rc;
  h.S = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sbytes * nfg))) return rc;
  h.G = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sbytes))) return rc;
  h.ghat = (c2*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(double) * 2 * nparts))) return rc;
  h.part = (double*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(uint64_t) * d.max_iter))) return rc;
  h.norms = (uint64_t*)p;
  if ((rc = dalloc(I.allocs, &p, 64))) return rc;
  h.iter_base = (int32_t*)p;
  h.flags = (int32_t*)p + 1;
  c2* tw = nullptr;
  if ((rc = get_twiddles(ctx, I.nx, &tw))) return rc;
  h.tw_x = tw;
  if ((rc = get_twiddles(ctx, I.ny, &tw))) return rc;
  h.tw_y = tw;
  h.tw_z = nullptr;
  if (I.nz > 1) {
    if ((rc = get_twiddles(ctx, I.nz, &tw))) return rc;
    h.tw_z = tw;
  }
  if ((rc = dalloc(I.allocs, &p, sizeof(InstDev)))) return rc;
  I.dev = (InstDev*)p;
  if ((rc = dalloc(I.allocs, &p, sizeof(InstDev*)))) return rc;
  I.d_solo = (InstDev**)p;
  HIPCHK(hipMemcpy(I.d_solo, &I.dev, sizeof(InstDev*), hipMemcpyHostToDevice));
  // No instance iterates before its first setup: park the iteration base
  // beyond the cap so every iteration kernel exits at once.
  int32_t init[2] = {d.max_iter + 1, 0};
  HIPCHK(hipMemcpy(h.iter_base, init, sizeof(init), hipMemcpyHostToDevice));
  HIPCHK(hipMemset(h.norms, 0, sizeof(uint64_t) * d.max_iter));
  return PFCH_OK;
}

int launch(const void* f, dim3 g, dim3 b, size_t lds, void** args, hipStream_t s) {
  HIPCHK(hipLaunchKernel(f, g, b, args, lds, s));
  return PFCH_OK;
}

// The iteration kernels of a group in launch order: 2D {column, row}; 3D
// {y forward, z, y inverse, row}.
struct Stage {
  const void* f;
  int bpi;
  dim3 block;
  size_t lds;
};
// Grid of a stage launched for `nm` instances: one block per item.
unsigned stage_grid(const Stage& st, unsigned nm) { return nm * (unsigned)st.bpi; }
int iter_stages(const Group& G, Stage* st) {
  if (G.ndim == 3) {
    st[0] = Stage{G.y3.fwd, G.y3_bpi, G.y3_block, G.y3_lds};
    st[1] = Stage{G.z3.iter, G.z3_bpi, G.z3_block, G.z3_lds};
    st[2] = Stage{G.y3.inv, G.y3_bpi, G.y3_block, G.y3_lds};
    st[3] = Stage{G.rk.iter, G.row_bpi, G.row_block, G.row_lds};
    return 4;
  }
  st[0] = Stage{G.ck.iter, G.col_bpi, G.col_block, G.col_lds};
  st[1] = Stage{G.rk.iter, G.row_bpi, G.row_block, G.row_lds};
  return 2;
}

// Build (once per chunk length) a graph running `K` iterations of every
// group, then the chunk-end bookkeeping.
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
  for (auto& G : ctx->groups) {
    hipGraphNode_t prev = nullptr;
    const unsigned nm = (unsigned)G.members.size();
    Stage st[4];
    const int ns = iter_stages(G, st);
    for (int l = 0; l < K; ++l) {
      for (int k = 0; k < ns; ++k) {
        hipKernelNodeParams p{};
        InstDev** grp = G.d_members;
        int bpi = st[k].bpi;
        int lv = l;
        int total = (int)nm * bpi;
        void* args[] = {&grp, &bpi, &lv, &total};
        p.func = const_cast<void*>(st[k].f);
        p.gridDim = dim3(stage_grid(st[k], nm));
        p.blockDim = st[k].block;
        p.sharedMemBytes = (unsigned)st[k].lds;
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
    uint32_t* dseq = ctx->d_seq;
    uint32_t* hseq = nullptr;
    HIPCHK(hipHostGetDevicePointer((void**)&hseq, ctx->h_seq, 0));
    void* args[] = {&ptrs, &n, &k, &dseq, &hseq};
    p.func = (void*)&k_chunk_end;
    p.gridDim = dim3(1);
    p.blockDim = dim3(chunk_end_threads(k, n));
    p.sharedMemBytes = 0;
    p.kernelParams = args;
    hipGraphNode_t node;
    HIPCHK(hipGraphAddKernelNode(&node, g, tails.data(), tails.size(), &p));
    // accept of the instances whose set-up published a destination
    hipKernelNodeParams q{};
    double** nodsts = nullptr;
    double* part = ctx->d_part;
    AccDsts none{};
    int check = 2;
    void* qargs[] = {&ptrs, &nodsts, &part, &none, &check};
    q.func = (void*)&k_accept;
    q.gridDim = dim3(ctx->acc_blocks, n);
    q.blockDim = dim3(ACC_THREADS);
    q.sharedMemBytes = 0;
    q.kernelParams = qargs;
    hipGraphNode_t anode;
    HIPCHK(hipGraphAddKernelNode(&anode, g, &node, 1, &q));
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
// further chunks are short.  Every length up to 32 has its own graph (the
// common iteration counts, built when first needed); longer ones are
// rounded to a small set.
int chunk_len(int want) {
  if (want <= 32) return want < 1 ? 1 : want;
  static const int lens[] = {40, 48, 56, 64};
  for (int k : lens)
    if (k >= want) return k;
  return 64;
}

struct StepSetup {
  const double* un;
  const double* unm1;
  const double* xin;
  double a, b, c, theta, rho;
  double* acc_dst = nullptr;
  const double* lun = nullptr;
  const double* lunm1 = nullptr;
  double* acc_ldst = nullptr;
};

StepArgs to_args(const StepSetup& ss) {
  StepArgs sa{};
  sa.un = ss.un;
  sa.unm1 = ss.unm1 ? ss.unm1 : ss.un;
  sa.xin = ss.xin;
  sa.rho = ss.rho;
  sa.a = ss.a;
  sa.theta = ss.theta;
  sa.gu = ss.b - ss.a * (1.0 - ss.theta) / ss.theta;
  sa.gm = ss.c;
  sa.acc_dst = ss.acc_dst;
  sa.lun = ss.lun;
  sa.lunm1 = ss.lunm1;
  sa.acc_ldst = ss.acc_ldst;
  return sa;
}

// Coefficients (eq. obj:BDF2 with backward Euler first, eq. obj:MP) and
// extrapolation factor for the next step of size dt.
StepSetup step_setup_for(const Instance& I, double dt) {
  StepSetup ss{};
  ss.un = I.U[I.ucur];
  ss.unm1 = I.has_prev ? I.U[1 - I.ucur] : I.U[I.ucur];
  ss.xin = nullptr;
  if (scheme_mp(I.d.scheme)) {
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

// Setup kernels for `nm` instances of group G described by the device arrays
// (grp, args).
// start_fch: some instance takes Delta x0 from transforms (k_row_setup,
// k_row_start_fch); lap: some instance takes it from kept Laplacians
// (k_row_setup_lap).  Each row set-up kernel skips the other's instances.
// 2D groups without the transform path of the FCH set-up (PFC, and FCH
// from kept Laplacians) launch no column set-up: the step's first column
// iteration transforms g and sums the averaged-Newton partials itself.
bool setup_folds(const Group& G, bool start_fch) { return G.ndim == 2 && (G.model != PFCH_FCH || !start_fch); }

// A device array `args` must already carry fold = setup_folds(G, start_fch).
// allow_fold = false keeps the column set-up (kernel timing: the iteration
// kernels then run without the folded set-up work).
int launch_setup(pfch_ctx* ctx, const Group& G, InstDev** grp, StepArgs* args, unsigned nm,
                 const StepArgsInline* inl = nullptr, bool start_fch = true, bool lap = false,
                 bool allow_fold = true) {
  int rc;
  int rbpi = G.srow_bpi, cbpi = G.scol_bpi;
  const bool fold = allow_fold && setup_folds(G, start_fch);
  StepArgsInline il{};
  if (inl) {
    il = *inl;
    for (unsigned k = 0; k < nm; ++k) il.a[k].fold = fold ? 1 : 0;
    args = nullptr;
  }
  if (start_fch || G.model != PFCH_FCH) {
    void* a[] = {&grp, &args, &rbpi, &il};
    if ((rc = launch(G.rs.setup, dim3(nm * rbpi), G.srow_block, G.srow_lds, a, ctx->stream))) return rc;
  }
  if (lap && G.model == PFCH_FCH) {
    void* a[] = {&grp, &args, &rbpi, &il};
    if (G.rs.setup_lap_fp && rbpi == G.rows / 2) {  // one row pair per block: one partial-sum slot each
      const size_t lds = (size_t)G.rs.setup_fp_elems * sizeof(c2);
      if ((rc = launch(G.rs.setup_lap_fp, dim3(nm * rbpi), dim3(4 * G.rs.T), lds, a, ctx->stream))) return rc;
    } else if ((rc = launch(G.rs.setup_lap, dim3(nm * rbpi), G.srow_block, G.srow_lds, a, ctx->stream))) {
      return rc;
    }
  }
  if (G.ndim == 3) {
    int ybpi = G.y3_bpi, zbpi = G.z3_bpi;
    void* a[] = {&grp, &ybpi};
    if ((rc = launch(G.y3.setup, dim3(nm * ybpi), G.y3_block, G.y3_lds, a, ctx->stream))) return rc;
    void* b[] = {&grp, &zbpi};
    if ((rc = launch(G.z3.setup, dim3(nm * zbpi), G.z3_block, G.z3_lds, b, ctx->stream))) return rc;
    return PFCH_OK;
  }
  if (!fold) {
    void* a[] = {&grp, &cbpi};
    if ((rc = launch(G.cs.setup, dim3(nm * cbpi), G.scol_block, G.scol_lds, a, ctx->stream))) return rc;
  }
  if (G.model == PFCH_FCH && start_fch) {
    void* a[] = {&grp, &rbpi};
    if ((rc = launch(G.rs.start_fch, dim3(nm * rbpi), G.srow_block, G.srow_lds, a, ctx->stream))) return rc;
  }
  return PFCH_OK;
}

int launch_setup_solo(pfch_ctx* ctx, Instance& I, const StepSetup& ss, bool allow_fold = true) {
  StepArgsInline inl{};
  inl.a[0] = to_args(ss);
  return launch_setup(ctx, ctx->groups[I.group], I.d_solo, nullptr, 1, &inl, ss.lun == nullptr,
                      ss.lun != nullptr, allow_fold);
}

// Park instances (all of them when insts is the context's array) so that
// later chunk graphs neither iterate nor accept for them.
int launch_park(pfch_ctx* ctx, InstDev** insts, int n) {
  void* a[] = {&insts, &n};
  return launch((const void*)&k_park, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, a, ctx->stream);
}

// Discard a set-up queued by the previous pfch_step.  That set-up marked
// every instance's record running and published its accept destination
// (the u^{n-1} slot), so the next chunk graph, replayed for whichever
// instances a later call solves, would otherwise iterate every instance and
// copy its solution over its history: the instances are parked on the
// device first, in stream order behind the queued set-up.
int drop_spec(pfch_ctx* ctx) {
  if (!ctx->spec) return PFCH_OK;
  ctx->spec = false;
  return launch_park(ctx, ctx->d_ptrs, (int)ctx->inst.size());
}

int launch_accept(pfch_ctx* ctx, AccDsts inl, double** dsts, double* part, int check) {
  InstDev** ptrs = ctx->d_ptrs;
  void* a[] = {&ptrs, &dsts, &part, &inl, &check};
  return launch((const void*)&k_accept, dim3(ctx->acc_blocks, (unsigned)ctx->inst.size()), dim3(ACC_THREADS), 0, a,
                ctx->stream);
}

// Wait for chunk number `want`: watch the pinned counter the chunk-end kernel
// writes (a chunk takes tens of microseconds; a stream synchronisation would
// add its own wake-up latency), then fall back to synchronising the stream,
// which also reports any error.  Work queued after the chunk (the graph's
// accept) keeps running in stream order.
int wait_chunk(pfch_ctx* ctx, uint32_t want) {
  const volatile uint32_t* seq = ctx->h_seq;
  for (long k = 0; k < 2000000; ++k) {  // bounded: about a millisecond or more
    if ((int32_t)(*seq - want) >= 0) {
      // the stop records written before the counter are read after it
      std::atomic_thread_fence(std::memory_order_acquire);
      return PFCH_OK;
    }
#if defined(__x86_64__)
    __builtin_ia32_pause();
#endif
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

// Copy the mirrored stop records of chunk `want` into ctx->recs.  Each
// mirror carries the number of the chunk that wrote it, written after its
// other fields; a mirror from an earlier chunk is not used: the stream is
// synchronised (the chunk has then ended) and the mirrors read again.  A
// mirror that still carries another number is an internal error.
int take_records(pfch_ctx* ctx, uint32_t want) {
  const int n = (int)ctx->inst.size();
  ctx->recs.resize(n);
  for (int pass = 0; pass < 2; ++pass) {
    bool all = true;
    for (int i = 0; i < n; ++i) {
      const volatile StopRec* h = ctx->h_recs + i;
      const uint32_t tag = h->seq;
      std::atomic_thread_fence(std::memory_order_acquire);
      if (tag != want) {
        all = false;
        continue;
      }
      StopRec r{};
      r.stop_iter = h->stop_iter;
      r.flags = h->flags;
      r.norm_bits = h->norm_bits;
      r.seq = tag;
      ctx->recs[i] = r;
    }
    if (all) return PFCH_OK;
    if (pass == 0) {
      HIPCHK(hipStreamSynchronize(ctx->stream));
      const char* dbg = std::getenv("PFCH_DEBUG");
      if (dbg && dbg[0] && dbg[0] != '0')
        std::fprintf(stderr, "pfch: stop records behind chunk %u; read again after synchronising\n", want);
    }
  }
  return PFCH_E_INTERNAL;
}

// Replay iteration chunks until every instance in `active` has stopped.  The
// chunk graph ends with the stop records mirrored into pinned host memory and
// a progress counter the host waits on, then the accept of instances whose
// set-up published a destination.
int run_iterations(pfch_ctx* ctx, const std::vector<int>& active) {
  int predicted = 1;
  bool known = true;
  for (int i : active) {
    predicted = std::max(predicted, ctx->inst[i].last_iters);
    known = known && ctx->inst[i].last_iters > 0;
  }
  int K = chunk_len(known ? predicted : 16);
  for (;;) {
    hipGraphExec_t ex;
    int rc = get_graph(ctx, K, &ex);
    if (rc) return rc;
    HIPCHK(hipGraphLaunch(ex, ctx->stream));
    if ((rc = wait_chunk(ctx, ++ctx->seq))) return rc;
    if ((rc = take_records(ctx, ctx->seq))) return rc;
    bool all = true;
    for (int i : active) {
      const StopRec& r = ctx->recs[i];
      if (r.stop_iter < 0 && !(r.flags & FLAG_PRECOND)) all = false;
    }
    if (all) return PFCH_OK;
    K = chunk_len(2);
  }
}

// The host's decision on a final stop record (Alg. 2's stopping rule, the
// iteration cap, a non-finite norm, the preconditioner check).  A record
// still marked running is never a result.
int stop_status(int32_t stop_iter, int32_t flags, uint64_t norm_bits, int32_t max_iter, int* iters,
                double* dnorm) {
  const double nv = double_of(norm_bits);
  *dnorm = nv;
  *iters = 0;
  if (flags & FLAG_PRECOND) return PFCH_E_PRECOND;
  if (stop_iter < 0) {
    *dnorm = NAN;
    return PFCH_E_INTERNAL;
  }
  if (stop_iter >= max_iter) {
    *iters = max_iter;
    return PFCH_E_NOCONV;
  }
  *iters = stop_iter + 1;
  if (!std::isfinite(nv)) return PFCH_E_NONFINITE;
  return PFCH_OK;
}

int status_of(const Instance& I, const StopRec& r, int* iters, double* dnorm) {
  return stop_status(r.stop_iter, r.flags, r.norm_bits, I.d.max_iter, iters, dnorm);
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
  if (I.h.imex) {
    const double e2 = I.d.eps * I.d.eps;
    out[1] = I.h.imex_b0;
    out[2] = I.h.imex_b2;
    out[3] = I.d.model == PFCH_PFC ? 1.0 : e2 * e2;
    return PFCH_OK;
  }
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

// Gate of the learned guess.  The network's correction is used while the
// least-squares gain fitted to it on the step before stays at LG_GAIN_ON or
// above; a lower gain means the correction has stopped predicting the
// solutions (it over-predicts them), and measured iteration counts rise
// then even with the correction scaled down by the gain.  Such a step
// leaves the correction out (gain 0, on the device), and the instance then
// takes the extrapolated guess (the paper's, with no network call) for
// LG_PROBE_AFTER << min(failed probes, 3) fixed-size steps before it probes
// the network again: the first probe step adds the correction with gain 0
// (its guess is the extrapolation), the second the gain fitted to the
// first if that reaches LG_GAIN_ON, which also decides the gate.
constexpr double LG_GAIN_ON = 0.98;
constexpr int LG_PROBE_AFTER = 16;

// The gain of an instance's learned correction back to 1 (after a new
// history or network), the gate open.
int reset_gain(pfch_ctx* ctx, Instance& I) {
  static const double one[2] = {1.0, 1.0};
  I.gain_ready = false;
  I.gain_fresh = false;
  I.lg_off = false;
  I.lg_wait = 0;
  I.lg_probe = 0;
  I.lg_fails = 0;
  I.gain_par = 0;
  if (I.gbuf) HIPCHK(hipMemcpyAsync(I.gbuf, one, sizeof(one), hipMemcpyHostToDevice, ctx->stream));
  return PFCH_OK;
}

// Learned initial guesses of the instances `ids` (extrapolation factors
// rho[k]): network inputs from (u^n, u^{n-1}) (resampled to the network's
// grid when it is coarser), one forward pass per network and batch of up to
// its max_batch instances, then per instance x0 = extrapolation +
// g Pi_0(so * y) (y interpolated back to the instance's grid) into
// I.xguess, g the instance's gain: 1 after pfch_set_state or pfch_set_fno,
// then after every fixed-size step that took the learned guess the least
// squares gain of that step's correction against the solution it reached,
// clamped to [0, 1]; all on the context's stream.
int learned_guesses(pfch_ctx* ctx, const std::vector<int>& ids, const std::vector<double>& rho) {
  hipStream_t s = ctx->stream;
  std::vector<char> done(ids.size(), 0);
  for (size_t a = 0; a < ids.size(); ++a) {
    if (done[a]) continue;
    pfch_fno* net = ctx->inst[ids[a]].fno;
    Fno& F = net->f;
    std::vector<size_t> chunk;
    for (size_t b = a; b < ids.size() && (int)chunk.size() < F.maxb; ++b)
      if (!done[b] && ctx->inst[ids[b]].fno == net) {
        chunk.push_back(b);
        done[b] = 1;
      }
    // batch slots ordered by fine grid, so that the resampling products of
    // the instances on one fine grid are one batched call per stage
    std::stable_sort(chunk.begin(), chunk.end(), [&](size_t x, size_t y) {
      return (uintptr_t)ctx->inst[ids[x]].fno_rs < (uintptr_t)ctx->inst[ids[y]].fno_rs;
    });
    std::vector<char> gain_from(chunk.size(), 0);  // slot k: the gain from its last step's partials
    // runs[r] = (first slot, count) of instances sharing one resampler (or none)
    std::vector<std::pair<size_t, size_t>> runs;
    for (size_t k = 0; k < chunk.size(); ++k)
      if (k == 0 || ctx->inst[ids[chunk[k]]].fno_rs != ctx->inst[ids[chunk[k - 1]]].fno_rs)
        runs.push_back({k, 1});
      else
        ++runs.back().second;
    for (const auto& run : runs) {
      Resampler* R = ctx->inst[ids[chunk[run.first]]].fno_rs;
      for (size_t j = 0; j < run.second; ++j) {
        const size_t k = run.first + j;
        Instance& I = ctx->inst[ids[chunk[k]]];
        const double* nrm = I.fno_norm;
        const long long P = I.npts;
        float* dst = R ? R->Xf + (long long)j * 2 * P : F.xin + (long long)k * 2 * F.P;
        // with the inputs, the previous step's guess (still in xguess) against
        // the solution it reached (now u^n): partials of that step's gain
        const bool gp = I.gain_ready;
        gain_from[k] = gp ? 1 : 0;
        I.gain_ready = false;
        I.gain_fresh = gp;
        hipLaunchKernelGGL(k_guess_inputs, dim3(GUESS_BLOCKS), dim3(256), 0, s, (const double*)I.U[1 - I.ucur],
                           (const double*)I.U[I.ucur], P, nrm[0], nrm[1], nrm[2], dst,
                           gp ? (const double*)I.xguess : nullptr, gp ? (const float*)I.gcor : nullptr,
                           I.gbuf + 2);
      }
      if (R && resample_down(F, *R, R->Xf, 2, F.xin + (long long)run.first * 2 * F.P, (int)run.second, s) !=
                   hipSuccess)
        return PFCH_E_HIP;
    }
    if (fno_forward(F, F.xin, (int)chunk.size(), s) != hipSuccess) return PFCH_E_HIP;
    for (const auto& run : runs) {
      Resampler* R = ctx->inst[ids[chunk[run.first]]].fno_rs;
      if (R && resample_up(F, *R, F.y + (long long)run.first * F.P, (int)run.second, s) != hipSuccess)
        return PFCH_E_HIP;
    }
    for (size_t k = 0; k < chunk.size(); ++k) {
      Instance& I = ctx->inst[ids[chunk[k]]];
      const long long P = I.npts;
      const float* y = F.y + (long long)k * F.P;
      if (I.fno_rs) {
        size_t first = k;
        while (first > 0 && ctx->inst[ids[chunk[first - 1]]].fno_rs == I.fno_rs) --first;
        y = I.fno_rs->yf + (long long)(k - first) * P;
      }
      hipLaunchKernelGGL(k_guess_ysum, dim3(GUESS_BLOCKS), dim3(256), 0, s, y, P, I.gpart);
      hipLaunchKernelGGL(k_guess_scalars, dim3(1), dim3(256), 0, s, I.gpart, P, (const double*)I.gbuf + I.gain_par,
                         gain_from[k] ? (const double*)I.gbuf + 2 : nullptr, LG_GAIN_ON, I.gbuf + (1 - I.gain_par),
                         ctx->d_gain + ids[chunk[k]]);
      hipLaunchKernelGGL(k_learned_guess, dim3(std::min(blocks_for(P / 2), 4096u)), dim3(256), 0, s,
                         (const double*)I.U[I.ucur], (const double*)I.U[1 - I.ucur], rho[chunk[k]], I.fno_norm[3],
                         y, (const double*)I.gpart + GUESS_BLOCKS, (const double*)I.gbuf + (1 - I.gain_par), P,
                         I.xguess, I.gcor);
      I.gain_par ^= 1;
    }
    HIPCHK(hipGetLastError());
  }
  return PFCH_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: per (model, scheme, Nx, Ny), the radix schedule and launch
// geometry of the two iteration kernels are picked by timing every candidate
// on the group's first instance (from a zero state; the iteration kernels'
// cost does not depend on the values).  Choices are kept for the process.
// PFCH_AUTOTUNE=0 in the environment keeps the defaults.
// ---------------------------------------------------------------------------
struct TuneChoice {
  int row_alt = -1, teams = 0;  // alt -1: default plan
  int col_alt = -1, cb = 0;
  int cy = 0, kyb = 0;          // 3D: y-pass columns per block, z-pass ky per block
  int y3_alt = -1, z3_alt = -1;  // 3D: y- and z-pass plans
};

std::mutex& tune_mutex() {
  static std::mutex m;
  return m;
}
std::map<std::tuple<int, int, int, int, int>, TuneChoice>& tune_cache() {
  static std::map<std::tuple<int, int, int, int, int>, TuneChoice> c;
  return c;
}

bool autotune_enabled() {
  const char* e = std::getenv("PFCH_AUTOTUNE");
  return !(e && e[0] == '0');
}

constexpr size_t LDS_MAX = 160 * 1024;
// An alternative replaces the default only when it is clearly faster, so
// that timing noise does not flip the choice between processes.
constexpr float TUNE_MARGIN = 0.94f;

bool row_geometry_ok(const Group& G, const RowK& k, int teams) {
  const int pairs = G.rows / 2;
  return k.T * teams <= 256 && pairs % teams == 0 && ((size_t)teams * k.lds_elems + k.tw_elems) * sizeof(c2) <= LDS_MAX;
}
bool col_geometry_ok(const Group& G, const ColK& k, int cb) {
  const int H = G.nx / 2;
  if (k.fp && cb != 1) return false;  // field-parallel: one column per block
  return k.T * cb <= 512 && H % cb == 0 && ((size_t)cb * k.lds_elems + k.tw_elems) * sizeof(c2) <= LDS_MAX;
}

void apply_row(Group& G, const RowK& k, int teams) {
  G.rk = k;
  G.row_block = dim3(k.T * teams);
  G.row_bpi = (G.rows / 2) / teams;
  G.row_lds = ((size_t)teams * k.lds_elems + k.tw_elems) * sizeof(c2);
  if (G.row_lds > 65536)
    (void)hipFuncSetAttribute(k.iter, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.row_lds);
}
void apply_col(Group& G, const ColK& k, int cb) {
  G.ck = k;
  G.col_block = dim3(k.T * cb);
  G.col_bpi = (G.nx / 2) / cb;
  G.col_lds = ((size_t)cb * k.lds_elems + k.tw_elems) * sizeof(c2);
  if (G.col_lds > 65536)
    (void)hipFuncSetAttribute(k.iter, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.col_lds);
}

// Milliseconds per launch of one iteration stage on instance I alone.
int time_stage(pfch_ctx* ctx, Instance& I, const Stage& st, hipEvent_t e0, hipEvent_t e1, float* ms) {
  InstDev** grp = I.d_solo;
  int bpi = st.bpi;
  int l0 = 0;
  int total = bpi;
  void* a[] = {&grp, &bpi, &l0, &total};
  const dim3 grid(stage_grid(st, 1));
  constexpr int WARM = 2, REPS = 8, ROUNDS = 3;
  int rc;
  for (int r = 0; r < WARM; ++r)
    if ((rc = launch(st.f, grid, st.block, st.lds, a, ctx->stream))) return rc;
  float best = 0.f;
  for (int round = 0; round < ROUNDS; ++round) {  // best of three batches
    HIPCHK(hipEventRecord(e0, ctx->stream));
    for (int r = 0; r < REPS; ++r)
      if ((rc = launch(st.f, grid, st.block, st.lds, a, ctx->stream))) return rc;
    HIPCHK(hipEventRecord(e1, ctx->stream));
    HIPCHK(hipEventSynchronize(e1));
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e0, e1));
    if (round == 0 || t < best) best = t;
  }
  *ms = best / REPS;
  return PFCH_OK;
}

// The group's current row (which = 1) or column (which = 0) kernel.
int time_iter_kernel(pfch_ctx* ctx, const Group& G, Instance& I, int which, hipEvent_t e0, hipEvent_t e1,
                     float* ms) {
  Stage st[4];
  iter_stages(G, st);
  return time_stage(ctx, I, st[which], e0, e1, ms);
}

bool y3_geometry_ok(const Group& G, const Y3K& k, int cy) {
  return (cy == 1 || cy == 2 || cy == 4) && cy * k.T <= 512 && ((size_t)cy * k.lds_elems + k.tw_elems) * sizeof(c2) <= LDS_MAX;
}
bool z3_geometry_ok(const Group& G, const Z3K& k, int kyb) {
  return kyb >= 1 && (kyb & (kyb - 1)) == 0 && TW * kyb * k.T <= 512 && G.ny % kyb == 0 &&
         2 * kyb <= G.ny && ((size_t)TW * kyb * k.lds_elems + k.tw_elems) * sizeof(c2) <= LDS_MAX;
}
void apply_y3(Group& G, const Y3K& k, int cy) {
  G.y3 = k;
  G.y3_block = dim3(G.y3.T * cy);
  G.y3_bpi = G.nz * (G.nx / 2) / cy;
  G.y3_lds = ((size_t)cy * G.y3.lds_elems + G.y3.tw_elems) * sizeof(c2);
  const void* fs[] = {G.y3.fwd, G.y3.inv, G.y3.setup, G.y3.rhs_fwd, G.y3.rhs_inv};
  for (const void* f : fs)
    if (G.y3_lds > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.y3_lds);
}
void apply_z3(Group& G, const Z3K& k, int kyb) {
  G.z3 = k;
  G.z3_block = dim3(G.z3.T * TW * kyb);
  G.z3_bpi = (G.nx / 2 / TW) * (G.ny / kyb);
  G.z3_lds = ((size_t)TW * kyb * G.z3.lds_elems + G.z3.tw_elems) * sizeof(c2);
  const void* fs[] = {G.z3.iter, G.z3.setup, G.z3.rhs};
  for (const void* f : fs)
    if (G.z3_lds > 65536) (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.z3_lds);
}

// A choice the group's kernels can run: alternatives in range, geometry
// within the launch and LDS limits.
bool choice_ok(const Group& G, const TuneChoice& c) {
  if (c.row_alt < -1 || c.row_alt >= (int)G.ralts.size()) return false;
  const RowK& rk = c.row_alt < 0 ? G.rs : G.ralts[c.row_alt];
  if (c.teams < 1 || (c.teams & (c.teams - 1)) || !row_geometry_ok(G, rk, c.teams)) return false;
  if (G.ndim == 3) {
    if (c.y3_alt < -1 || c.y3_alt >= (int)G.y3alts.size() || c.z3_alt < -1 || c.z3_alt >= (int)G.z3alts.size())
      return false;
    return y3_geometry_ok(G, c.y3_alt < 0 ? G.y3d : G.y3alts[c.y3_alt], c.cy) &&
           z3_geometry_ok(G, c.z3_alt < 0 ? G.z3d : G.z3alts[c.z3_alt], c.kyb);
  }
  if (c.col_alt < -1 || c.col_alt >= (int)G.calts.size()) return false;
  const ColK& ck = c.col_alt < 0 ? G.cs : G.calts[c.col_alt];
  if (c.cb != 1 && c.cb != 2 && c.cb != 4) return false;
  return col_geometry_ok(G, ck, c.cb);
}

// Tuning file: with PFCH_TUNE_FILE set, a choice recorded there for the
// group's (model, scheme, Nx, Ny, Nz) is used instead of timing, and a new
// choice is appended.  One line per entry:
//   model scheme nx ny nz  row_alt teams col_alt cb 0 cy kyb y3_alt z3_alt
// (the last valid line for a key wins; the tenth field is reserved and must
// be 0).
using TuneKey = std::tuple<int, int, int, int, int>;

bool tune_file_lookup(const TuneKey& key, TuneChoice* out) {
  const char* path = std::getenv("PFCH_TUNE_FILE");
  if (!path || !path[0]) return false;
  FILE* f = std::fopen(path, "r");
  if (!f) return false;
  char line[256];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    int v[14];
    if (std::sscanf(line, "%d %d %d %d %d %d %d %d %d %d %d %d %d %d", &v[0], &v[1], &v[2], &v[3], &v[4], &v[5],
                    &v[6], &v[7], &v[8], &v[9], &v[10], &v[11], &v[12], &v[13]) != 14)
      continue;
    if (std::make_tuple(v[0], v[1], v[2], v[3], v[4]) != key || v[9] != 0) continue;
    TuneChoice c;
    c.row_alt = v[5];
    c.teams = v[6];
    c.col_alt = v[7];
    c.cb = v[8];
    c.cy = v[10];
    c.kyb = v[11];
    c.y3_alt = v[12];
    c.z3_alt = v[13];
    *out = c;
    found = true;
  }
  std::fclose(f);
  return found;
}

void tune_file_store(const TuneKey& key, const TuneChoice& c) {
  const char* path = std::getenv("PFCH_TUNE_FILE");
  if (!path || !path[0]) return;
  FILE* f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%d %d %d %d %d  %d %d %d %d %d %d %d %d %d\n", std::get<0>(key), std::get<1>(key), std::get<2>(key),
               std::get<3>(key), std::get<4>(key), c.row_alt, c.teams, c.col_alt, c.cb, 0, c.cy,
               c.kyb, c.y3_alt, c.z3_alt);
  std::fclose(f);
}

void apply_choice(Group& G, const TuneChoice& c) {
  apply_row(G, c.row_alt < 0 ? G.rs : G.ralts[c.row_alt], c.teams);
  if (G.ndim == 3) {
    apply_y3(G, c.y3_alt < 0 ? G.y3d : G.y3alts[c.y3_alt], c.cy);
    apply_z3(G, c.z3_alt < 0 ? G.z3d : G.z3alts[c.z3_alt], c.kyb);
  } else {
    apply_col(G, c.col_alt < 0 ? G.cs : G.calts[c.col_alt], c.cb);
  }
}

// 3D groups: rows per block of the x-pass, columns per block of the
// y-passes (both timed on the forward pass) and ky per block of the z-pass.
int tune_group3(pfch_ctx* ctx, Group& G, TuneChoice& best) {
  Instance& I = ctx->inst[G.members[0]];
  const size_t bytes = sizeof(double) * (size_t)I.npts;
  HIPCHK(hipMemsetAsync(I.U[0], 0, bytes, ctx->stream));
  HIPCHK(hipMemsetAsync(I.U[1], 0, bytes, ctx->stream));
  I.has_prev = false;
  int rc;
  if ((rc = launch_setup_solo(ctx, I, step_setup_for(I, 1e-3), false))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  Stage st[4];
  float t_def = 0.f, t = 0.f;
  // x-pass
  iter_stages(G, st);
  if ((rc = time_stage(ctx, I, st[3], e0, e1, &t_def))) return rc;
  float t_best = t_def;
  for (int alt = -1; alt < (int)G.ralts.size(); ++alt) {
    const RowK& k = alt < 0 ? G.rs : G.ralts[alt];
    for (int teams = 1; teams <= 64; teams *= 2) {
      if (!row_geometry_ok(G, k, teams) || (alt < 0 && teams == best.teams)) continue;
      apply_row(G, k, teams);
      iter_stages(G, st);
      if ((rc = time_stage(ctx, I, st[3], e0, e1, &t))) return rc;
      if (t < TUNE_MARGIN * t_def && t < t_best) {
        t_best = t;
        best.row_alt = alt;
        best.teams = teams;
      }
    }
  }
  apply_row(G, best.row_alt < 0 ? G.rs : G.ralts[best.row_alt], best.teams);
  // y-passes (timed on the forward pass)
  iter_stages(G, st);
  if ((rc = time_stage(ctx, I, st[0], e0, e1, &t_def))) return rc;
  t_best = t_def;
  for (int alt = -1; alt < (int)G.y3alts.size(); ++alt) {
    const Y3K& k = alt < 0 ? G.y3d : G.y3alts[alt];
    for (int cy = 1; cy <= 4; cy *= 2) {
      if (!y3_geometry_ok(G, k, cy) || (alt < 0 && cy == best.cy)) continue;
      apply_y3(G, k, cy);
      iter_stages(G, st);
      if ((rc = time_stage(ctx, I, st[0], e0, e1, &t))) return rc;
      if (t < TUNE_MARGIN * t_def && t < t_best) {
        t_best = t;
        best.y3_alt = alt;
        best.cy = cy;
      }
    }
  }
  apply_y3(G, best.y3_alt < 0 ? G.y3d : G.y3alts[best.y3_alt], best.cy);
  // z-pass
  iter_stages(G, st);
  if ((rc = time_stage(ctx, I, st[1], e0, e1, &t_def))) return rc;
  t_best = t_def;
  for (int alt = -1; alt < (int)G.z3alts.size(); ++alt) {
    const Z3K& k = alt < 0 ? G.z3d : G.z3alts[alt];
    for (int kyb = 1; kyb <= 32; kyb *= 2) {
      if (!z3_geometry_ok(G, k, kyb) || (alt < 0 && kyb == best.kyb)) continue;
      apply_z3(G, k, kyb);
      iter_stages(G, st);
      if ((rc = time_stage(ctx, I, st[1], e0, e1, &t))) return rc;
      if (t < TUNE_MARGIN * t_def && t < t_best) {
        t_best = t;
        best.z3_alt = alt;
        best.kyb = kyb;
      }
    }
  }
  apply_z3(G, best.z3_alt < 0 ? G.z3d : G.z3alts[best.z3_alt], best.kyb);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return PFCH_OK;
}

int tune_group(pfch_ctx* ctx, Group& G, bool* used_instance) {
  *used_instance = false;
  if (!autotune_enabled()) return PFCH_OK;  // defaults as set up
  const auto key = std::make_tuple(G.model, G.scheme, G.nx, G.ny, G.nz);
  std::lock_guard<std::mutex> lock(tune_mutex());
  auto& cache = tune_cache();
  auto it = cache.find(key);
  if (it != cache.end()) {
    apply_choice(G, it->second);
    return PFCH_OK;
  }
  {
    TuneChoice fc;
    if (tune_file_lookup(key, &fc) && choice_ok(G, fc)) {
      apply_choice(G, fc);
      cache[key] = fc;
      return PFCH_OK;
    }
  }
  if (G.ndim == 3) {
    TuneChoice c;
    c.teams = (int)(G.row_block.x / G.rk.T);
    c.cy = (int)(G.y3_block.x / G.y3.T);
    c.kyb = (int)(G.z3_block.x / (G.z3.T * TW));
    *used_instance = true;
    int rc;
    if ((rc = tune_group3(ctx, G, c))) return rc;
    cache[key] = c;
    tune_file_store(key, c);
    return PFCH_OK;
  }
  TuneChoice def;
  def.teams = (int)(G.row_block.x / G.rk.T);
  def.cb = (int)(G.col_block.x / G.ck.T);
  if (G.ralts.empty() && G.calts.empty()) {
    cache[key] = def;
    return PFCH_OK;
  }
  Instance& I = ctx->inst[G.members[0]];
  *used_instance = true;
  const size_t bytes = sizeof(double) * (size_t)I.npts;
  HIPCHK(hipMemsetAsync(I.U[0], 0, bytes, ctx->stream));
  HIPCHK(hipMemsetAsync(I.U[1], 0, bytes, ctx->stream));
  I.has_prev = false;
  int rc;
  if ((rc = launch_setup_solo(ctx, I, step_setup_for(I, 1e-3), false))) return rc;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  TuneChoice best = def;
  float t_def_row = 0.f, t_def_col = 0.f;
  // rows
  {
    apply_row(G, G.rs, def.teams);
    if ((rc = time_iter_kernel(ctx, G, I, 1, e0, e1, &t_def_row))) return rc;
    float t_best = t_def_row;
    for (int alt = -1; alt < (int)G.ralts.size(); ++alt) {
      const RowK& k = alt < 0 ? G.rs : G.ralts[alt];
      for (int teams = 1; teams <= 64; teams *= 2) {
        if (!row_geometry_ok(G, k, teams) || (alt < 0 && teams == def.teams)) continue;
        apply_row(G, k, teams);
        float t = 0.f;
        if ((rc = time_iter_kernel(ctx, G, I, 1, e0, e1, &t))) return rc;
        if (t < TUNE_MARGIN * t_def_row && t < t_best) {
          t_best = t;
          best.row_alt = alt;
          best.teams = teams;
        }
      }
    }
  }
  // columns
  {
    apply_col(G, G.cs, def.cb);
    if ((rc = time_iter_kernel(ctx, G, I, 0, e0, e1, &t_def_col))) return rc;
    float t_best = t_def_col;
    for (int alt = -1; alt < (int)G.calts.size(); ++alt) {
      const ColK& k = alt < 0 ? G.cs : G.calts[alt];
      for (int cb = 1; cb <= 4; cb *= 2) {
        if (!col_geometry_ok(G, k, cb) || (alt < 0 && cb == def.cb)) continue;
        apply_col(G, k, cb);
        float t = 0.f;
        if ((rc = time_iter_kernel(ctx, G, I, 0, e0, e1, &t))) return rc;
        if (t < TUNE_MARGIN * t_def_col && t < t_best) {
          t_best = t;
          best.col_alt = alt;
          best.cb = cb;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  apply_choice(G, best);
  cache[key] = best;
  tune_file_store(key, best);
  return PFCH_OK;
}

int fft_pairs_of(const Instance& I, int iters) {
  // Transform pairs of real fields (one forward + one inverse 2D transform
  // of a real field counts as one pair).  Per iteration: PFC 2 forward + 1
  // inverse, FCH 3 forward + 2 inverse.  Setup: g (+ x0 and its Laplacian,
  // + u^n for the midpoint rule, FCH), plus the first iteration's forwards.
  const bool fch = I.d.model == PFCH_FCH;
  const int per_iter = fch ? 5 : 3;
  const int setup = fch ? (scheme_mp(I.d.scheme) ? 2 * 3 + 3 : 2 * 2 + 3) : 1 + 2;
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
    case PFCH_E_INTERNAL: return "internal error: a solve record was not final";
    case PFCH_E_SCRATCH: return "grid too large for the static scratch of the allocation-free entry point";
    default: return "unknown error";
  }
}

int pfch_stop_status(int32_t stop_iter, int32_t flags, uint64_t norm_bits, int32_t max_iter, int32_t* iters,
                     double* dnorm_inf) {
  if (!iters || !dnorm_inf || max_iter < 1) return PFCH_E_INVAL;
  int it = 0;
  double dn = 0.0;
  const int rc = stop_status(stop_iter, flags, norm_bits, max_iter, &it, &dn);
  *iters = it;
  *dnorm_inf = dn;
  return rc;
}

int pfch_validate_desc(const pfch_instance_desc* d) {
  if (!d) return PFCH_E_INVAL;
  if (d->model != PFCH_PFC && d->model != PFCH_FCH) return PFCH_E_INVAL;
  if (d->scheme < PFCH_BDF2 || d->scheme > PFCH_LMP) return PFCH_E_INVAL;
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
  if (d->n_eta < 0 || d->n_eta > 8) return PFCH_E_INVAL;
  for (int i = 0; i < d->n_eta; ++i)
    if (!(d->eta[i] >= 0.0) || !std::isfinite(d->eta[i])) return PFCH_E_INVAL;
  if (d->max_iter < 1 || d->max_iter > 1000000) return PFCH_E_INVAL;
  if (d->guess != 0 && d->guess != 1) return PFCH_E_INVAL;
  if (scheme_imex(d->scheme) && d->guess != 0) return PFCH_E_INVAL;  // no solve to warm-start
  if (d->ndim == 3) {
    // 3D: PFC, x length as in 2D, y and z lengths of the 3D passes
    if (d->model != PFCH_PFC) return PFCH_E_UNSUPPORTED;
    if (!supported_len(d->n[0]) || !supported_len3(d->n[1]) || !supported_len3(d->n[2]))
      return PFCH_E_UNSUPPORTED;
    return PFCH_OK;
  }
  if (!supported_len(d->n[0]) || !supported_len(d->n[1])) return PFCH_E_UNSUPPORTED;
  return PFCH_OK;
}

void pfch_destroy(pfch_ctx* ctx) {
  if (!ctx) return;
  // work queued by the last step (its accept copy) may still be running; the
  // null stream (0) is synchronised like any other
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : ctx->graph_defs) (void)hipGraphDestroy(g);
  for (auto& I : ctx->inst)
    for (void* p : I.allocs) (void)hipFree(p);
  for (void* p : ctx->allocs) (void)hipFree(p);
  for (void* p : ctx->host_allocs) (void)hipHostFree(p);
  delete ctx;
}

int pfch_create(const pfch_instance_desc* descs, int32_t n_inst, void* hip_stream, pfch_ctx** out) {
  if (!out || !descs || n_inst < 1) return PFCH_E_INVAL;
  *out = nullptr;
  for (int i = 0; i < n_inst; ++i) {
    int rc = pfch_validate_desc(&descs[i]);
    if (rc) return rc;
  }
  // the static scratch of pfch_rhs_noalloc on this device, resolved here so
  // that the entry point itself makes no runtime look-up
  int dev = -1;
  void* scr = nullptr;
  if (hipGetDevice(&dev) != hipSuccess) return PFCH_E_HIP;
  if (int rc0 = scratch_for_device(dev, &scr)) return rc0;
  auto ctx = new (std::nothrow) pfch_ctx();
  if (!ctx) return PFCH_E_NOMEM;
  ctx->device = dev;
  ctx->scratch = scr;
  ctx->stream = (hipStream_t)hip_stream;
  ctx->inst.resize(n_inst);
  int rc = PFCH_OK;
  void* p = nullptr;
  // --- groups by (model, scheme, Nx, Ny, Nz)
  std::map<std::tuple<int, int, int, int, int>, int> gidx;
  for (int i = 0; i < n_inst; ++i) {
    Instance& I = ctx->inst[i];
    I.d = descs[i];
    I.nx = I.d.n[0];
    I.ny = I.d.n[1];
    I.nz = I.d.ndim == 3 ? I.d.n[2] : 1;
    I.nh = I.nx / 2;
    I.rows = I.ny * I.nz;
    I.npts = (int64_t)I.nx * I.ny * I.nz;
    const int eff_scheme = scheme_mp(I.d.scheme) ? PFCH_MP : PFCH_BDF2;  // kernel variant
    auto key = std::make_tuple(I.d.model, eff_scheme, I.nx, I.ny, I.nz);
    auto it = gidx.find(key);
    if (it == gidx.end()) {
      Group G;
      G.model = I.d.model;
      G.scheme = eff_scheme;
      G.nx = I.nx;
      G.ny = I.ny;
      G.nz = I.nz;
      G.rows = I.rows;
      G.ndim = I.d.ndim;
      const bool mps = scheme_mp(I.d.scheme);
      bool ok;
      if (G.ndim == 3) {
        ok = (mps ? row_kernels<MODEL_PFC, true>(I.nx, G.rs) : row_kernels<MODEL_PFC, false>(I.nx, G.rs)) &&
             y3_kernels(I.ny, G.y3d) && z3_kernels(I.nz, G.z3d);
        G.y3 = G.y3d;
        G.z3 = G.z3d;
        if (mps)
          row_alternatives<MODEL_PFC, true>(I.nx, G.ralts);
        else
          row_alternatives<MODEL_PFC, false>(I.nx, G.ralts);
        y3_alternatives(I.ny, G.y3alts);
        z3_alternatives(I.nz, G.z3alts);
      } else if (G.model == PFCH_PFC) {
        ok = (mps ? row_kernels<MODEL_PFC, true>(I.nx, G.rs) : row_kernels<MODEL_PFC, false>(I.nx, G.rs)) &&
             col_kernels<MODEL_PFC>(I.ny, G.cs);
        if (mps)
          row_alternatives<MODEL_PFC, true>(I.nx, G.ralts);
        else
          row_alternatives<MODEL_PFC, false>(I.nx, G.ralts);
        col_alternatives<MODEL_PFC>(I.ny, G.calts);
        if (mps)
          row_fp_alternatives<MODEL_PFC, true>(I.nx, G.ralts);
        else
          row_fp_alternatives<MODEL_PFC, false>(I.nx, G.ralts);
        col_fp_alternatives<MODEL_PFC>(I.ny, G.calts);
      } else {
        ok = (mps ? row_kernels<MODEL_FCH, true>(I.nx, G.rs) : row_kernels<MODEL_FCH, false>(I.nx, G.rs)) &&
             col_kernels<MODEL_FCH>(I.ny, G.cs);
        if (mps)
          row_alternatives<MODEL_FCH, true>(I.nx, G.ralts);
        else
          row_alternatives<MODEL_FCH, false>(I.nx, G.ralts);
        col_alternatives<MODEL_FCH>(I.ny, G.calts);
        if (mps)
          row_fp_alternatives<MODEL_FCH, true>(I.nx, G.ralts);
        else
          row_fp_alternatives<MODEL_FCH, false>(I.nx, G.ralts);
        col_fp_alternatives<MODEL_FCH>(I.ny, G.calts);
      }
      G.rk = G.rs;
      G.ck = G.cs;
      if (!ok) {
        delete ctx;
        return PFCH_E_UNSUPPORTED;
      }
      it = gidx.emplace(key, (int)ctx->groups.size()).first;
      ctx->groups.push_back(G);
    }
    I.group = it->second;
    ctx->groups[I.group].members.push_back(i);
  }
  for (auto& G : ctx->groups) {
    const int nm = (int)G.members.size();
    const int pairs = G.rows / 2, H = G.nx / 2;
    const int teams = pick_teams(G.rs.T, pairs);
    G.srow_block = G.row_block = dim3(G.rs.T * teams);
    G.srow_bpi = G.row_bpi = pairs / teams;
    G.srow_lds = G.row_lds = ((size_t)teams * G.rs.lds_elems + G.rs.tw_elems) * sizeof(c2);
    if (G.ndim == 3) {
      // y-pass: the widest tile part (<= 512 threads); z-pass: 4 columns of
      // a tile times kyb consecutive ky (<= 512 threads, kyb <= Ny/2)
      int cy = 4;
      while (cy > 1 && cy * G.y3.T > 512) cy >>= 1;
      G.y3_block = dim3(G.y3.T * cy);
      G.y3_bpi = G.nz * H / cy;
      G.y3_lds = ((size_t)cy * G.y3.lds_elems + G.y3.tw_elems) * sizeof(c2);
      int kyb = 4;
      while (kyb > 1 && (TW * kyb * G.z3.T > 512 || G.ny % kyb != 0 || 2 * kyb > G.ny)) kyb >>= 1;
      G.z3_block = dim3(G.z3.T * TW * kyb);
      G.z3_bpi = (H / TW) * (G.ny / kyb);
      G.z3_lds = ((size_t)TW * kyb * G.z3.lds_elems + G.z3.tw_elems) * sizeof(c2);
      if (G.y3_lds > 160 * 1024 || G.z3_lds > 160 * 1024) {
        rc = PFCH_E_UNSUPPORTED;
        goto fail;
      }
      const void* ys[] = {G.y3.fwd, G.y3.inv, G.y3.setup, G.y3.rhs_fwd, G.y3.rhs_inv};
      for (const void* f : ys)
        if (G.y3_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.y3_lds);
      const void* zs[] = {G.z3.iter, G.z3.setup, G.z3.rhs};
      for (const void* f : zs)
        if (G.z3_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.z3_lds);
    } else {
      const int cb = pick_cols(G.cs.T, H);
      G.scol_block = G.col_block = dim3(G.cs.T * cb);
      G.scol_bpi = G.col_bpi = H / cb;
      G.scol_lds = G.col_lds = ((size_t)cb * G.cs.lds_elems + G.cs.tw_elems) * sizeof(c2);
    }
    if (G.row_lds > 160 * 1024 || G.col_lds > 160 * 1024) {
      rc = PFCH_E_UNSUPPORTED;
      goto fail;
    }
    if ((rc = dalloc(ctx->allocs, &p, sizeof(InstDev*) * nm))) goto fail;
    G.d_members = (InstDev**)p;
    if ((rc = dalloc(ctx->allocs, &p, sizeof(StepArgs) * nm))) goto fail;
    G.d_args = (StepArgs*)p;
    if ((rc = halloc(ctx->host_allocs, &p, sizeof(StepArgs) * nm))) goto fail;
    G.h_args = (StepArgs*)p;
    if ((rc = dalloc(ctx->allocs, &p, sizeof(double*) * 2 * nm))) goto fail;
    G.d_rptr = (const double**)p;
    if ((rc = halloc(ctx->host_allocs, &p, sizeof(double*) * 2 * nm))) goto fail;
    G.h_rptr = (const double**)p;
    if (G.ndim == 2) {
      const void* rr[] = {G.rs.rhs_fwd, G.rs.rhs_mid, G.rs.rhs_inv};
      for (const void* f : rr)
        if (f && G.srow_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.srow_lds);
      const void* rc2[] = {G.cs.rhs_lap, G.cs.rhs};
      for (const void* f : rc2)
        if (f && G.scol_lds > 65536)
          (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.scol_lds);
    }
    const void* fs[] = {G.rs.iter, G.rs.setup, G.rs.start_fch, G.rs.setup_lap};
    for (const void* f : fs)
      if (f && G.row_lds > 65536)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.row_lds);
    const void* gs[] = {G.cs.iter, G.cs.setup};
    for (const void* f : gs)
      if (f && G.col_lds > 65536)
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G.col_lds);
  }
  if ((rc = dalloc(ctx->allocs, &p, sizeof(StopRec) * n_inst))) goto fail;
  ctx->d_recs = (StopRec*)p;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(InstDev*) * n_inst))) goto fail;
  ctx->d_ptrs = (InstDev**)p;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(double*) * n_inst))) goto fail;
  ctx->d_dsts = (double**)p;
  for (int i = 0; i < n_inst; ++i)  // about two points per thread, at most ACC_BLOCKS blocks
    ctx->acc_blocks = std::max(ctx->acc_blocks,
                               (int)std::min<int64_t>(ACC_BLOCKS, (ctx->inst[i].npts + 2 * ACC_THREADS - 1) /
                                                                      (2 * ACC_THREADS)));
  if ((rc = dalloc(ctx->allocs, &p, sizeof(double) * n_inst * ACC_BLOCKS))) goto fail;
  ctx->d_part = (double*)p;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(double) * n_inst))) goto fail;
  ctx->d_scale = (double*)p;
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(StopRec) * n_inst, true))) goto fail;
  ctx->h_recs = (StopRec*)p;
  for (int i = 0; i < n_inst; ++i) ctx->h_recs[i].stop_iter = -1;  // not stopped until a chunk says so
  ctx->recs.assign(n_inst, StopRec{-1, 0, 0, 0, 0});
  if ((rc = halloc(ctx->host_allocs, &p, 64))) goto fail;
  ctx->h_scratch = (int32_t*)p;
  if ((rc = halloc(ctx->host_allocs, &p, 64, true))) goto fail;
  ctx->h_seq = (uint32_t*)p;
  *ctx->h_seq = 0;
  if ((rc = dalloc(ctx->allocs, &p, 64))) goto fail;
  ctx->d_seq = (uint32_t*)p;
  if (hipMemset(ctx->d_seq, 0, 64) != hipSuccess) {
    rc = PFCH_E_HIP;
    goto fail;
  }
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(double*) * n_inst))) goto fail;
  ctx->h_dsts = (double**)p;
  // coherent: the mass kernel writes the pinned buffer directly
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(double) * n_inst, true))) goto fail;
  ctx->h_mass = (double*)p;
  if (hipHostGetDevicePointer((void**)&ctx->d_mass, ctx->h_mass, 0) != hipSuccess) {
    rc = PFCH_E_HIP;
    goto fail;
  }
  // coherent too: the learned-guess kernel writes each instance's gain here
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(double) * n_inst, true))) goto fail;
  ctx->h_gain = (double*)p;
  if (hipHostGetDevicePointer((void**)&ctx->d_gain, ctx->h_gain, 0) != hipSuccess) {
    rc = PFCH_E_HIP;
    goto fail;
  }
  if ((rc = dalloc(ctx->allocs, &p, sizeof(EstArgs) * n_inst))) goto fail;
  ctx->d_est = (EstArgs*)p;
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(EstArgs) * n_inst))) goto fail;
  ctx->h_est = (EstArgs*)p;
  if ((rc = dalloc(ctx->allocs, &p, sizeof(double) * 2 * EST_BLOCKS * n_inst))) goto fail;
  ctx->d_est_part = (double*)p;
  if ((rc = halloc(ctx->host_allocs, &p, sizeof(double) * 2 * EST_BLOCKS * n_inst))) goto fail;
  ctx->h_est_part = (double*)p;
  {
    std::vector<InstDev*> ptrs(n_inst);
    std::vector<double> scale(n_inst);
    for (int i = 0; i < n_inst; ++i) {
      Instance& I = ctx->inst[i];
      if ((rc = setup_instance(ctx, I, ctx->groups[I.group].srow_bpi))) goto fail;
      I.h.rec = ctx->d_recs + i;
      {
        void* hp = nullptr;
        if (hipHostGetDevicePointer(&hp, ctx->h_recs, 0) != hipSuccess) {
          rc = PFCH_E_HIP;
          goto fail;
        }
        I.h.rec_host = (StopRec*)hp + i;
      }
      if (hipMemcpy(I.dev, &I.h, sizeof(InstDev), hipMemcpyHostToDevice) != hipSuccess) {
        rc = PFCH_E_HIP;
        goto fail;
      }
      ptrs[i] = I.dev;
      scale[i] = 1.0 / (double)I.npts;
    }
    if (hipMemcpy(ctx->d_ptrs, ptrs.data(), sizeof(InstDev*) * n_inst, hipMemcpyHostToDevice) !=
            hipSuccess ||
        hipMemcpy(ctx->d_scale, scale.data(), sizeof(double) * n_inst, hipMemcpyHostToDevice) !=
            hipSuccess) {
      rc = PFCH_E_HIP;
      goto fail;
    }
    for (auto& G : ctx->groups) {
      std::vector<InstDev*> mp;
      for (int i : G.members) mp.push_back(ctx->inst[i].dev);
      if (hipMemcpy(G.d_members, mp.data(), sizeof(InstDev*) * mp.size(), hipMemcpyHostToDevice) !=
          hipSuccess) {
        rc = PFCH_E_HIP;
        goto fail;
      }
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
    // autotune the iteration kernels, then return the instances it used to
    // the state of a fresh context (no iteration pending)
    bool any = false;
    for (auto& G : ctx->groups) {
      bool used = false;
      if ((rc = tune_group(ctx, G, &used))) goto fail;
      if (used) {
        Instance& I = ctx->inst[G.members[0]];
        int32_t park = I.d.max_iter + 1;
        if (hipMemcpy(I.h.iter_base, &park, sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess) {
          rc = PFCH_E_HIP;
          goto fail;
        }
        any = true;
      }
    }
    if (any && hipMemcpy(ctx->d_recs, recs.data(), sizeof(StopRec) * n_inst, hipMemcpyHostToDevice) !=
                   hipSuccess) {
      rc = PFCH_E_HIP;
      goto fail;
    }
  }
  *out = ctx;
  return PFCH_OK;
fail:
  pfch_destroy(ctx);
  return rc;
}

int pfch_set_stats_detail(pfch_ctx* ctx, int32_t detail) {
  if (!ctx || detail < 0 || detail > 2) return PFCH_E_INVAL;
  if (detail == 2) {  // the residual needs u^{n-1} after the accept has replaced it
    for (auto& I : ctx->inst) {
      if (I.uprobe) continue;
      void* p = nullptr;
      int rc = dalloc(I.allocs, &p, sizeof(double) * (size_t)I.npts);
      if (rc) return rc;
      I.uprobe = (double*)p;
    }
  }
  ctx->stats_detail = detail;
  return PFCH_OK;
}

}  // extern "C"

namespace {

// HIP-event timing of the iteration kernels of the instances `members` (all
// of group G; grp is their device pointer array in that order), launched
// together as the solve launches them: `reps` solves of the step of size dt
// from their current states, an event pair on every launch; out[k] = the
// average microseconds of stage k over the iterations in which every member
// still worked.  The members' states are not changed; their iteration
// workspaces are, and they are parked afterwards.
int time_iterations(pfch_ctx* ctx, Group& G, InstDev** grp, const std::vector<int>& members, double dt, int reps,
                    double out[5]) {
  const unsigned nm = (unsigned)members.size();
  Stage st[4];
  const int ns = iter_stages(G, st);
  // iterations launched per solve: the largest last count plus two
  int last = 1, cap = 1 << 30;
  for (int i : members) {
    last = std::max(last, ctx->inst[i].last_iters);
    cap = std::min(cap, ctx->inst[i].d.max_iter);
  }
  const int nit = std::min(cap, last + 2);
  std::vector<hipEvent_t> ev((size_t)2 * ns * nit);
  for (auto& e : ev) HIPCHK(hipEventCreate(&e));
  std::vector<uint64_t> norms((size_t)nm * nit);
  double sum[4] = {0, 0, 0, 0};
  int cnt[4] = {0, 0, 0, 0};
  int work = nit;  // iterations in which every member worked (the same in every solve)
  double chain_sum = 0.0;
  int chain_cnt = 0;
  int rc = PFCH_OK;
  // reps solves with an event pair on every launch, then reps solves with one
  // event before the first launch and one after the last working iteration
  for (int r = 0; r < 2 * reps && rc == PFCH_OK; ++r) {
    const bool chained = r >= reps;
    if (chained && work < 1) break;
    if (nm == 1) {
      if ((rc = launch_setup_solo(ctx, ctx->inst[members[0]], step_setup_for(ctx->inst[members[0]], dt), false)))
        break;
    } else {
      for (unsigned k = 0; k < nm; ++k) {
        G.h_args[k] = to_args(step_setup_for(ctx->inst[members[k]], dt));
        G.h_args[k].fold = 0;  // the column set-up runs: the iteration kernels are timed alone
      }
      if (hipMemcpyAsync(G.d_args, G.h_args, sizeof(StepArgs) * nm, hipMemcpyHostToDevice, ctx->stream) !=
          hipSuccess) {
        rc = PFCH_E_HIP;
        break;
      }
      if ((rc = launch_setup(ctx, G, grp, G.d_args, nm, nullptr, true, false, false))) break;
    }
    for (int j = 0; j < nit && rc == PFCH_OK; ++j) {
      if (chained && j == 0 && hipEventRecord(ev[0], ctx->stream) != hipSuccess) rc = PFCH_E_HIP;
      for (int k = 0; k < ns && rc == PFCH_OK; ++k) {
        int bpi = st[k].bpi, lv = j, total = (int)nm * bpi;
        void* a[] = {&grp, &bpi, &lv, &total};
        hipEvent_t* e = &ev[2 * ((size_t)j * ns + k)];
        if (hipExtLaunchKernel(st[k].f, dim3(stage_grid(st[k], nm)), st[k].block, a, st[k].lds, ctx->stream,
                               chained ? nullptr : e[0], chained ? nullptr : e[1], 0) != hipSuccess)
          rc = PFCH_E_HIP;
      }
      if (chained && j == work - 1 && rc == PFCH_OK && hipEventRecord(ev[1], ctx->stream) != hipSuccess)
        rc = PFCH_E_HIP;
    }
    if (rc) break;
    for (unsigned k = 0; k < nm && rc == PFCH_OK; ++k)
      if (hipMemcpyAsync(norms.data() + (size_t)k * nit, ctx->inst[members[k]].h.norms, sizeof(uint64_t) * nit,
                         hipMemcpyDeviceToHost, ctx->stream) != hipSuccess)
        rc = PFCH_E_HIP;
    if (rc || hipStreamSynchronize(ctx->stream) != hipSuccess) {
      rc = PFCH_E_HIP;
      break;
    }
    if (chained) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, ev[0], ev[1]) == hipSuccess) {
        chain_sum += 1e3 * t / work;
        chain_cnt += 1;
      }
      continue;
    }
    // iteration j did work for every member if j = 0 or no member stopped at j-1
    int j = 0;
    for (; j < nit; ++j) {
      bool all = true;
      for (unsigned k = 0; k < nm && j > 0; ++k) {
        const uint64_t b = norms[(size_t)k * nit + j - 1];
        if (b < ctx->inst[members[k]].h.tol_bits || b >= INF_BITS) all = false;
      }
      if (!all) break;
      for (int k = 0; k < ns; ++k) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, ev[2 * ((size_t)j * ns + k)], ev[2 * ((size_t)j * ns + k) + 1]) != hipSuccess)
          continue;
        sum[k] += 1e3 * t;
        cnt[k] += 1;
      }
    }
    work = std::min(work, j);
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (rc) return rc;
  for (int k = 0; k < 4; ++k) out[k] = cnt[k] ? sum[k] / cnt[k] : 0.0;
  out[4] = chain_cnt ? chain_sum / chain_cnt : 0.0;
  // park the members so that later chunk launches leave them alone
  if ((rc = launch_park(ctx, grp, (int)nm))) return rc;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

}  // namespace

extern "C" {

int pfch_time_kernels(pfch_ctx* ctx, double dt, int32_t reps, double out[5]) {
  if (!ctx || !out || reps < 1 || !(dt > 0.0) || !std::isfinite(dt)) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Instance& I = ctx->inst[0];
  return time_iterations(ctx, ctx->groups[I.group], I.d_solo, std::vector<int>{0}, dt, reps, out);
}

int pfch_time_group(pfch_ctx* ctx, int32_t inst, double dt, int32_t reps, double out[5]) {
  if (!ctx || !out || inst < 0 || inst >= (int)ctx->inst.size() || reps < 1 || !(dt > 0.0) || !std::isfinite(dt))
    return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Group& G = ctx->groups[ctx->inst[inst].group];
  return time_iterations(ctx, G, G.d_members, G.members, dt, reps, out);
}

int pfch_time_kernels_events(pfch_ctx* ctx, double dt, int32_t reps, double out[4]) {
  if (!ctx || !out || reps < 1 || !(dt > 0.0) || !std::isfinite(dt)) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Instance& I = ctx->inst[0];
  const Group& G = ctx->groups[I.group];
  int rc;
  if ((rc = launch_setup_solo(ctx, I, step_setup_for(I, dt), false))) return rc;
  Stage st[4];
  const int ns = iter_stages(G, st);
  hipEvent_t e[5];
  for (auto& ev : e) HIPCHK(hipEventCreate(&ev));
  InstDev** grp = I.d_solo;
  int l0 = 0;  // iteration 0 after setup: every launch does full work
  HIPCHK(hipEventRecord(e[0], ctx->stream));
  for (int k = 0; k < ns; ++k) {
    int bpi = st[k].bpi;
    int total = bpi;
    void* a[] = {&grp, &bpi, &l0, &total};
    for (int r = 0; r < reps; ++r)
      if ((rc = launch(st[k].f, dim3(stage_grid(st[k], 1)), st[k].block, st[k].lds, a, ctx->stream))) return rc;
    HIPCHK(hipEventRecord(e[k + 1], ctx->stream));
  }
  HIPCHK(hipEventSynchronize(e[ns]));
  for (int k = 0; k < 4; ++k) out[k] = 0.0;
  for (int k = 0; k < ns; ++k) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, e[k], e[k + 1]));
    out[k] = 1e3 * t / reps;
  }
  for (auto& ev : e) (void)hipEventDestroy(ev);
  // park the instance so later chunk launches leave it alone
  int32_t* park = ctx->h_scratch;
  *park = I.d.max_iter + 1;
  HIPCHK(hipMemcpyAsync(I.h.iter_base, park, sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

int pfch_get_launch_config(pfch_ctx* ctx, int32_t inst, int64_t out[6]) {
  if (!ctx || !out || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  const Group& G = ctx->groups[ctx->inst[inst].group];
  const int64_t nm = (int64_t)G.members.size();
  out[0] = nm * G.row_bpi;
  out[1] = G.row_block.x;
  out[2] = (int64_t)G.row_lds;
  out[3] = nm * G.col_bpi;
  out[4] = G.col_block.x;
  out[5] = (int64_t)G.col_lds;
  return PFCH_OK;
}

int pfch_get_plan(pfch_ctx* ctx, int32_t inst, int32_t out[37]) {
  if (!ctx || !out || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  const Group& G = ctx->groups[ctx->inst[inst].group];
  auto find = [](const auto& alts, const void* f, auto get) {
    for (int k = 0; k < (int)alts.size(); ++k)
      if (get(alts[k]) == f) return k;
    return -1;
  };
  for (int k = 0; k < 37; ++k) out[k] = 0;  // out[36]: reserved
  out[0] = find(G.ralts, G.rk.iter, [](const RowK& k) { return k.iter; });
  out[1] = G.rk.T > 0 ? (int32_t)(G.row_block.x / G.rk.T) : 0;
  out[8] = (int32_t)G.ralts.size();
  for (int p = 0; p < 8; ++p) out[12 + p] = G.rk.radix[p];
  if (G.ndim == 3) {
    out[2] = -1;
    out[4] = find(G.y3alts, G.y3.fwd, [](const Y3K& k) { return k.fwd; });
    out[5] = (int32_t)(G.y3_block.x / G.y3.T);
    out[6] = find(G.z3alts, G.z3.iter, [](const Z3K& k) { return k.iter; });
    out[7] = (int32_t)(G.z3_block.x / (G.z3.T * TW));
    out[10] = (int32_t)G.y3alts.size();
    out[11] = (int32_t)G.z3alts.size();
    for (int p = 0; p < 8; ++p) {
      out[20 + p] = G.y3.radix[p];
      out[28 + p] = G.z3.radix[p];
    }
  } else {
    out[2] = find(G.calts, G.ck.iter, [](const ColK& k) { return k.iter; });
    out[3] = (int32_t)(G.col_block.x / G.ck.T);
    out[4] = out[6] = -1;
    out[9] = (int32_t)G.calts.size();
    for (int p = 0; p < 8; ++p) out[20 + p] = G.ck.radix[p];
  }
  return PFCH_OK;
}

int pfch_set_plan(pfch_ctx* ctx, int32_t inst, const int32_t choice[9]) {
  if (!ctx || !choice || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Group& G = ctx->groups[ctx->inst[inst].group];
  TuneChoice c;
  c.row_alt = choice[0];
  c.teams = choice[1];
  c.col_alt = choice[2];
  c.cb = choice[3];
  c.y3_alt = choice[4];
  c.cy = choice[5];
  c.z3_alt = choice[6];
  c.kyb = choice[7];
  if (choice[8] != 0 || !choice_ok(G, c)) return PFCH_E_INVAL;  // choice[8]: reserved
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (auto& kv : ctx->graphs) (void)hipGraphExecDestroy(kv.second);
  for (auto g : ctx->graph_defs) (void)hipGraphDestroy(g);
  ctx->graphs.clear();
  ctx->graph_defs.clear();
  apply_choice(G, c);
  return PFCH_OK;
}

int pfch_set_state(pfch_ctx* ctx, int32_t inst, const double* u_n, const double* u_nm1, double t,
                   double dt_prev, int32_t step_index) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !u_n) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  if (u_nm1 && !(dt_prev > 0.0)) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  const size_t bytes = sizeof(double) * (size_t)I.npts;
  HIPCHK(hipMemcpyAsync(I.U[I.ucur], u_n, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  if (u_nm1) HIPCHK(hipMemcpyAsync(I.U[1 - I.ucur], u_nm1, bytes, hipMemcpyDeviceToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  I.has_prev = u_nm1 != nullptr;
  I.t = t;
  I.dt_prev = u_nm1 ? dt_prev : 0.0;
  I.step_index = step_index;
  I.hist = I.has_prev ? 2 : 1;
  I.r_valid = false;
  I.lap_levels = 0;
  return reset_gain(ctx, I);
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

namespace {

// Outcome of the tentative solves of one step of every instance.
struct SolveOut {
  std::vector<int> status, iters, guess;
  std::vector<double> dn, a;
};

// The fused set-up (one row kernel doing four transforms, the column set-up
// folded into the first column iteration) is faster than the three-kernel
// path at every supported row length once its register use allows two waves
// per SIMD (g is transformed on its own, before x0 and v_breve are formed:
// 236 registers at 2048, 302 when they were all live at once).  Combined
// FCH 1024^2 + 2048^2 + PFC 192^3 set, batched: 68.5 -> 69.3 time-steps/s
// with the Laplacians kept at 2048 too, although the accept then also
// copies the Laplacian.
bool lap_history_pays(const Instance& I) { return I.nx <= 2048; }

// FCH with an extrapolated guess and two kept Laplacians: the set-up takes
// Delta x0 from them instead of from transforms of x0.
void lap_from_history(const Instance& I, StepSetup& ss) {
  if (I.dU[0] && lap_history_pays(I) && I.lap_levels >= 2 && I.has_prev && !ss.xin) {
    ss.lun = I.dU[I.ucur];
    ss.lunm1 = I.dU[1 - I.ucur];
  }
}

// Set-up of every instance's tentative solve at step size dt[i] (guess,
// averaged-Newton constants, transforms that start iteration 0); o gets the
// guess kind and a of each instance and empty results.
int launch_step_setups(pfch_ctx* ctx, const double* dt, SolveOut& o, bool accept) {
  const int n = (int)ctx->inst.size();
  o.status.assign(n, PFCH_OK);
  o.iters.assign(n, 0);
  o.guess.assign(n, 0);  // 0 extrapolated, 1 learned, 2 learned then extrapolated
  o.dn.assign(n, 0.0);
  o.a.assign(n, 0.0);
  int rc;
  // the learned guesses first: one network call per batch of instances
  std::vector<int> lids;
  std::vector<double> lrho;
  for (int i = 0; i < n; ++i) {
    const Instance& I = ctx->inst[i];
    if (I.fno && I.d.guess == 1 && I.has_prev && !I.lg_off) {
      lids.push_back(i);
      lrho.push_back(step_setup_for(I, dt[i]).rho);
      o.guess[i] = 1;
    }
  }
  if (!lids.empty() && (rc = learned_guesses(ctx, lids, lrho))) return rc;
  for (auto& G : ctx->groups) {
    for (size_t k = 0; k < G.members.size(); ++k) {
      Instance& I = ctx->inst[G.members[k]];
      StepSetup ss = step_setup_for(I, dt[G.members[k]]);
      if (accept) {
        ss.acc_dst = I.U[1 - I.ucur];
        if (lap_history_pays(I)) ss.acc_ldst = I.dU[1 - I.ucur];
      }
      if (o.guess[G.members[k]] == 1) ss.xin = I.xguess;
      lap_from_history(I, ss);
      o.a[G.members[k]] = ss.a;
      G.h_args[k] = to_args(ss);
    }
    const unsigned nm = (unsigned)G.members.size();
    bool start_fch = false, lap = false;
    for (unsigned k = 0; k < nm; ++k) {
      start_fch = start_fch || !G.h_args[k].lun;
      lap = lap || G.h_args[k].lun;
    }
    if (nm <= (unsigned)STEP_ARGS_INLINE) {
      StepArgsInline inl{};
      for (unsigned k = 0; k < nm; ++k) inl.a[k] = G.h_args[k];
      if ((rc = launch_setup(ctx, G, G.d_members, nullptr, nm, &inl, start_fch, lap))) return rc;
    } else {
      for (unsigned k = 0; k < nm; ++k) G.h_args[k].fold = setup_folds(G, start_fch) ? 1 : 0;
      HIPCHK(hipMemcpyAsync(G.d_args, G.h_args, sizeof(StepArgs) * nm, hipMemcpyHostToDevice,
                            ctx->stream));
      if ((rc = launch_setup(ctx, G, G.d_members, G.d_args, nm, nullptr, start_fch, lap))) return rc;
    }
  }
  return PFCH_OK;
}

// PAGD iterations of every instance after launch_step_setups, and the
// learned-guess fallback.  Nothing is accepted here (in-graph accepts of
// the set-up's published destinations aside).
int finish_solve(pfch_ctx* ctx, const double* dt, SolveOut& o, bool accept) {
  const int n = (int)ctx->inst.size();
  std::vector<int> active(n);
  int rc;
  for (int i = 0; i < n; ++i) active[i] = i;
  if ((rc = run_iterations(ctx, active))) return rc;
  // A learned guess that does not lead to convergence falls back to the
  // extrapolated guess: the step is solved again from it.
  std::vector<int> retry;
  for (int i = 0; i < n; ++i) {
    if (o.guess[i] != 1) continue;
    int it = 0;
    double d = 0.0;
    if (status_of(ctx->inst[i], ctx->recs[i], &it, &d) == PFCH_OK) continue;
    Instance& I = ctx->inst[i];
    StepSetup ss = step_setup_for(I, dt[i]);
    if (accept) {
      ss.acc_dst = I.U[1 - I.ucur];
      if (lap_history_pays(I)) ss.acc_ldst = I.dU[1 - I.ucur];
    }
    lap_from_history(I, ss);
    if ((rc = launch_setup_solo(ctx, I, ss))) return rc;
    o.guess[i] = 2;
    retry.push_back(i);
  }
  if (!retry.empty() && (rc = run_iterations(ctx, retry))) return rc;
  for (int i = 0; i < n; ++i) o.status[i] = status_of(ctx->inst[i], ctx->recs[i], &o.iters[i], &o.dn[i]);
  return PFCH_OK;
}

// Tentative solve of every instance at step size dt[i]: set-up, PAGD
// iterations, and the learned-guess fallback.  Nothing is accepted.
int solve_all(pfch_ctx* ctx, const double* dt, SolveOut& o, bool accept = false) {
  ctx->spec = false;  // every instance's set-up follows: a queued one needs no parking
  int rc;
  if ((rc = launch_step_setups(ctx, dt, o, accept))) return rc;
  return finish_solve(ctx, dt, o, accept);
}

// The converged iterate of instance I after solve_all; null unless the
// record is a final, converged one.
const double* solution_of(const Instance& I, const StopRec& r) {
  int it = 0;
  double dn = 0.0;
  if (status_of(I, r, &it, &dn) != PFCH_OK) return nullptr;
  return I.h.X[(r.stop_iter + 1) % 3];
}

// Accept the tentative solutions of the instances with take[i]: u^{n+1}
// into the history (with u^{n-2} kept for the adaptive estimators), time
// and step counters advanced; with want_mass, the mean of each accepted
// solution lands in ctx->h_mass after the stream is synchronised.
int accept_solutions(pfch_ctx* ctx, const std::vector<char>& take, const double* dt, const SolveOut& o,
                     bool want_mass, bool adaptive, bool copied = false) {
  const int n = (int)ctx->inst.size();
  int rc;
  if (!copied) {  // else the checked accept inside the chunk graph has copied them
    for (int i = 0; i < n; ++i) {
      Instance& I = ctx->inst[i];
      ctx->h_dsts[i] = nullptr;
      if (!take[i]) continue;
      if (adaptive) std::swap(I.Um2, I.U[1 - I.ucur]);  // u^{n-1} becomes u^{n-2}
      ctx->h_dsts[i] = I.U[1 - I.ucur];
    }
    AccDsts inl{};
    double** dsts = nullptr;
    if (n <= ACC_INLINE) {
      for (int i = 0; i < n; ++i) inl.p[i] = ctx->h_dsts[i];
    } else {
      HIPCHK(hipMemcpyAsync(ctx->d_dsts, ctx->h_dsts, sizeof(double*) * n, hipMemcpyHostToDevice, ctx->stream));
      dsts = ctx->d_dsts;
    }
    if ((rc = launch_accept(ctx, inl, dsts, want_mass ? ctx->d_part : nullptr, 0))) return rc;
  }
  if (want_mass) {
    const double* part = ctx->d_part;
    int nb = ctx->acc_blocks, nn = n;
    const double* scale = ctx->d_scale;
    double* o2 = ctx->d_mass;
    void* a[] = {&part, &nb, &nn, &scale, &o2};
    // written straight into the pinned host buffer (read after the stream
    // is synchronised)
    if ((rc = launch((const void*)&k_sum_parts, dim3(n), dim3(256), 0, a, ctx->stream))) return rc;
  }
  for (int i = 0; i < n; ++i) {
    if (!take[i]) continue;
    Instance& I = ctx->inst[i];
    I.ucur = 1 - I.ucur;
    if (adaptive) {
      I.dt_nm1 = I.dt_prev;
      I.hist = std::min(I.hist + 1, 3);
    } else {
      I.hist = 2;  // u^{n-2} is not kept by plain steps
      I.r_valid = false;
    }
    // the in-graph accept of pfch_step also keeps the Laplacian (FCH)
    I.lap_levels = copied && I.dU[0] && lap_history_pays(I) ? std::min(I.lap_levels + 1, 2) : 0;
    I.has_prev = true;
    I.dt_prev = dt[i];
    I.t += dt[i];
    I.step_index += 1;
    I.last_iters = o.iters[i];
  }
  return PFCH_OK;
}

int fill_stats(pfch_ctx* ctx, const SolveOut& o, int i, bool want_mass, bool accepted, pfch_stats& s) {
  Instance& I = ctx->inst[i];
  std::memset(&s, 0, sizeof(s));
  s.status = o.status[i];
  s.iters = o.iters[i];
  s.dnorm_inf = o.dn[i];
  s.fft_pairs = fft_pairs_of(I, o.iters[i]);
  s.guess = o.guess[i];
  s.mass = (want_mass && accepted) ? ctx->h_mass[i] : NAN;
  s.rnorm_inf = NAN;
  s.gain = o.guess[i] == 1 ? ctx->h_gain[i] : NAN;
  if (ctx->stats_detail > 0) {
    int rc = betas_host(ctx, I, o.a[i], s.beta);
    if (rc) return rc;
  } else {
    for (double& b : s.beta) b = NAN;
  }
  return PFCH_OK;
}

// Coefficients of a step of size dt from instance I's current history.
struct Coef {
  double a, b, c, theta;
};
Coef coef_of(const Instance& I, double dt) {
  const StepSetup ss = step_setup_for(I, dt);
  return Coef{ss.a, ss.b, ss.c, ss.theta};
}

// ||r(x)||_inf, r = -G'(x) of the step problem with coefficients k and
// history (un, unm1): the step set-up from x with the residual flag, then
// one iteration of the instance's iteration kernels, whose preconditioner is
// then the identity, so that the first norm slot holds ||r(x)||_inf.  Uses
// the instance's iteration workspaces (not its state); the instance is
// parked afterwards.  Synchronises the stream.  NaN for the IMEX schemes.
int residual_norm(pfch_ctx* ctx, Instance& I, const double* x, const double* un, const double* unm1,
                  const Coef& k, double* out) {
  *out = NAN;
  if (scheme_imex(I.d.scheme)) return PFCH_OK;
  StepSetup ss{};
  ss.un = un;
  ss.unm1 = unm1 ? unm1 : un;
  ss.xin = x;
  ss.a = k.a;
  ss.b = k.b;
  ss.c = k.c;
  ss.theta = k.theta;
  ss.rho = 0.0;
  StepArgsInline inl{};
  inl.a[0] = to_args(ss);
  inl.a[0].resid = 1;
  const Group& G = ctx->groups[I.group];
  int rc;
  if ((rc = launch_setup(ctx, G, I.d_solo, nullptr, 1, &inl, true, false))) return rc;
  Stage st[4];
  const int ns = iter_stages(G, st);
  InstDev** grp = I.d_solo;
  for (int q = 0; q < ns; ++q) {
    int bpi = st[q].bpi, l = 0, total = bpi;
    void* a[] = {&grp, &bpi, &l, &total};
    if ((rc = launch(st[q].f, dim3(stage_grid(st[q], 1)), st[q].block, st[q].lds, a, ctx->stream))) return rc;
  }
  if ((rc = launch_park(ctx, I.d_solo, 1))) return rc;
  uint64_t* bits = reinterpret_cast<uint64_t*>(ctx->h_scratch);
  HIPCHK(hipMemcpyAsync(bits, I.h.norms, sizeof(uint64_t), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  *out = double_of(*bits);
  return PFCH_OK;
}

// R(v) = M Delta mu(v) for the members of group G with a non-null src[k]
// (device field of member k) into dst[k].  Uses the members' spectral
// workspaces.
// The kernels of R(v) for the nm members of G: sources ps[k], destinations
// pd[k] (device arrays of nm pointers), spectral workspace `spec` (null: each
// instance's own).
int rhs_kernels(pfch_ctx* ctx, Group& G, InstDev** grp, unsigned nm, const double** ps, double** pd,
                c2* spec) {
  int rbpi = G.srow_bpi, cbpi = G.scol_bpi, rc;
  const dim3 rg(nm * rbpi), cg(nm * cbpi);
  {
    void* a[] = {&grp, &ps, &rbpi, &spec};
    if ((rc = launch(G.rs.rhs_fwd, rg, G.srow_block, G.srow_lds, a, ctx->stream))) return rc;
  }
  if (G.ndim == 3) {  // PFC: y forward, z (symbol and inverse), y inverse, then the rows
    int ybpi = G.y3_bpi, zbpi = G.z3_bpi;
    void* y[] = {&grp, &ps, &ybpi, &spec};
    void* z[] = {&grp, &ps, &zbpi, &spec};
    if ((rc = launch(G.y3.rhs_fwd, dim3(nm * ybpi), G.y3_block, G.y3_lds, y, ctx->stream))) return rc;
    if ((rc = launch(G.z3.rhs, dim3(nm * zbpi), G.z3_block, G.z3_lds, z, ctx->stream))) return rc;
    if ((rc = launch(G.y3.rhs_inv, dim3(nm * ybpi), G.y3_block, G.y3_lds, y, ctx->stream))) return rc;
    void* a[] = {&grp, &pd, &rbpi, &spec};
    return launch(G.rs.rhs_inv, rg, G.srow_block, G.srow_lds, a, ctx->stream);
  }
  if (G.model == PFCH_FCH) {
    void* a[] = {&grp, &ps, &cbpi, &spec};
    if ((rc = launch(G.cs.rhs_lap, cg, G.scol_block, G.scol_lds, a, ctx->stream))) return rc;
    void* b[] = {&grp, &ps, &rbpi, &spec};
    if ((rc = launch(G.rs.rhs_mid, rg, G.srow_block, G.srow_lds, b, ctx->stream))) return rc;
  }
  {
    void* a[] = {&grp, &ps, &cbpi, &spec};
    if ((rc = launch(G.cs.rhs, cg, G.scol_block, G.scol_lds, a, ctx->stream))) return rc;
  }
  {
    void* a[] = {&grp, &pd, &rbpi, &spec};
    if ((rc = launch(G.rs.rhs_inv, rg, G.srow_block, G.srow_lds, a, ctx->stream))) return rc;
  }
  return PFCH_OK;
}

int rhs_launch(pfch_ctx* ctx, Group& G, InstDev** grp, unsigned nm, const std::vector<const double*>& src,
               const std::vector<double*>& dst) {
  for (unsigned k = 0; k < nm; ++k) {
    G.h_rptr[k] = src[k];
    G.h_rptr[nm + k] = dst[k];
  }
  HIPCHK(hipMemcpyAsync(G.d_rptr, G.h_rptr, sizeof(double*) * 2 * nm, hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));  // the pinned staging is reused
  return rhs_kernels(ctx, G, grp, nm, G.d_rptr, (double**)(G.d_rptr + nm), nullptr);
}

// Buffers of the adaptive estimators, and R(u^n), R(u^{n-1}) of every
// instance whose history changed outside pfch_step_adaptive.
int prepare_adaptive(pfch_ctx* ctx) {
  int rc;
  void* p = nullptr;
  for (auto& I : ctx->inst) {
    if (I.Um2) continue;
    const size_t rbytes = sizeof(double) * (size_t)I.npts;
    if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
    I.Um2 = (double*)p;
    for (auto& r : I.R) {
      if ((rc = dalloc(I.allocs, &p, rbytes))) return rc;
      r = (double*)p;
    }
  }
  for (auto& G : ctx->groups) {
    const unsigned nm = (unsigned)G.members.size();
    for (int lev = 0; lev < 2; ++lev) {
      std::vector<const double*> src(nm, nullptr);
      std::vector<double*> dst(nm, nullptr);
      bool any = false;
      for (unsigned k = 0; k < nm; ++k) {
        Instance& I = ctx->inst[G.members[k]];
        if (I.r_valid || (lev == 1 && !I.has_prev)) continue;
        src[k] = lev == 0 ? I.U[I.ucur] : I.U[1 - I.ucur];
        dst[k] = I.R[lev];
        any = true;
      }
      if (any && (rc = rhs_launch(ctx, G, G.d_members, nm, src, dst))) return rc;
    }
  }
  for (auto& I : ctx->inst) {
    if (!I.r_valid) I.hist = I.has_prev ? 2 : 1;
    I.r_valid = true;
  }
  return PFCH_OK;
}

double next_dt(double err, double tol, double dt, double dt_min, double dt_max) {
  double bar;
  if (err == 0.0)
    bar = INFINITY;
  else if (std::isinf(err))
    bar = 0.0;
  else
    bar = 0.9 * std::cbrt(tol / err) * dt;
  return std::max(dt_min, std::min(bar, dt_max));
}

}  // namespace

int pfch_step(pfch_ctx* ctx, const double* dt, pfch_stats* st) {
  if (!ctx || !dt) return PFCH_E_INVAL;
  const int n = (int)ctx->inst.size();
  for (int i = 0; i < n; ++i)
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return PFCH_E_INVAL;
  SolveOut o;
  int rc;
  const bool want_mass = st && ctx->stats_detail > 0;
  const bool same_dt = (int)ctx->last_dt.size() == n && std::equal(dt, dt + n, ctx->last_dt.begin());
  // statistics detail 2: the residual of each solution afterwards needs this
  // step's coefficients and u^{n-1}, which the accept replaces
  const bool want_resid = st && ctx->stats_detail > 1;
  std::vector<Coef> coefs;
  if (want_resid) {
    coefs.resize(n);
    for (int i = 0; i < n; ++i) {
      Instance& I = ctx->inst[i];
      coefs[i] = coef_of(I, dt[i]);
      if (coefs[i].c != 0.0)
        HIPCHK(hipMemcpyAsync(I.uprobe, I.U[1 - I.ucur], sizeof(double) * (size_t)I.npts,
                              hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  // every instance's accept runs inside the chunk graph, checked on the
  // device against the same stop record the host reads afterwards
  if (ctx->spec && same_dt) {  // the set-up was enqueued by the previous call
    ctx->spec = false;
    o.status.assign(n, PFCH_OK);
    o.iters.assign(n, 0);
    o.dn.assign(n, 0.0);
    o.guess = ctx->spec_guess;
    o.a = ctx->spec_a;
    if ((rc = finish_solve(ctx, dt, o, true))) return rc;
  } else if ((rc = solve_all(ctx, dt, o, true))) {
    return rc;
  }
  int first_err = PFCH_OK;
  std::vector<char> take(n);
  for (int i = 0; i < n; ++i) {
    take[i] = o.status[i] == PFCH_OK;
    if (!take[i] && first_err == PFCH_OK) first_err = o.status[i];
  }
  if ((rc = accept_solutions(ctx, take, dt, o, want_mass, false, true))) return rc;
  if (st) {
    if (want_mass) HIPCHK(hipStreamSynchronize(ctx->stream));
    for (int i = 0; i < n; ++i)
      if ((rc = fill_stats(ctx, o, i, want_mass, take[i], st[i]))) return rc;
    for (int i = 0; i < n && want_resid; ++i) {
      if (!take[i]) continue;
      Instance& I = ctx->inst[i];  // accepted: u^{n+1} = U[ucur], u^n = U[1 - ucur]
      const double* un = I.U[1 - I.ucur];
      if ((rc = residual_norm(ctx, I, I.U[I.ucur], un, coefs[i].c != 0.0 ? I.uprobe : un, coefs[i],
                              &st[i].rnorm_inf)))
        return rc;
    }
  }
  // A loop at a fixed step size: enqueue the next step's set-up now, so that
  // it runs while control is with the caller.  Only when every instance
  // advanced.  A learned guess is formed then too (into the instance's own
  // guess buffer, in stream order, so later use of the network on this
  // stream does not change it).
  // the next learned guess may take this step's gain (learned guess taken
  // and accepted)
  for (int i = 0; i < n; ++i) ctx->inst[i].gain_ready = ctx->inst[i].gbuf && o.guess[i] == 1 && take[i];
  // the gate: a learned step whose gain was fitted to the step before it
  // closes it below LG_GAIN_ON (the gain is in pinned memory, written before
  // the solve that the host has waited for); closed, accepted steps count
  // down to the next probe
  for (int i = 0; i < n; ++i) {
    Instance& I = ctx->inst[i];
    if (!take[i] || !I.fno || I.d.guess != 1) continue;
    const bool fitted = o.guess[i] == 1 && I.gain_fresh;
    if (o.guess[i] == 2 || (fitted && !(ctx->h_gain[i] >= LG_GAIN_ON))) {
      // (guess 2: the learned guess did not lead to convergence)
      if (I.lg_probe > 0) ++I.lg_fails;
      I.lg_off = true;
      I.lg_wait = LG_PROBE_AFTER << std::min(I.lg_fails, 3);
      I.lg_probe = 0;
    } else if (o.guess[i] == 1) {
      if (fitted) I.lg_fails = 0;
      if (I.lg_probe > 0) --I.lg_probe;
    } else if (o.guess[i] == 0 && I.lg_off && --I.lg_wait <= 0) {
      I.lg_off = false;
      I.lg_probe = 2;
    }
  }
  const bool speculate = same_dt && first_err == PFCH_OK;
  ctx->last_dt.assign(dt, dt + n);
  if (speculate) {
    SolveOut nx;
    if ((rc = launch_step_setups(ctx, dt, nx, true))) return rc;
    ctx->spec = true;
    ctx->spec_guess = nx.guess;
    ctx->spec_a = nx.a;
  }
  return first_err;
}

int pfch_step_adaptive(pfch_ctx* ctx, const pfch_adapt_desc* ad, pfch_adapt_result* res) {
  if (!ctx || !ad || !res) return PFCH_E_INVAL;
  if (!(ad->tol > 0.0) || !std::isfinite(ad->tol) || !(ad->dt_min > 0.0) || !std::isfinite(ad->dt_max) ||
      !(ad->dt_max >= ad->dt_min) || ad->estimator < PFCH_EST_AUTO || ad->estimator > PFCH_EST_MIDAB2 ||
      ad->reserved != 0)
    return PFCH_E_INVAL;
  const int n = (int)ctx->inst.size();
  std::vector<double> dt(n);
  for (int i = 0; i < n; ++i) {
    dt[i] = res[i].dt_try;
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return PFCH_E_INVAL;
  }
  int rc;
  if ((rc = drop_spec(ctx))) return rc;  // instance state or workspaces change
  if ((rc = prepare_adaptive(ctx))) return rc;
  SolveOut o;
  if ((rc = solve_all(ctx, dt.data(), o))) return rc;
  for (auto& I : ctx->inst) I.gain_ready = false;  // accepts here do not feed the gain
  // R(u~) of every converged instance
  for (auto& G : ctx->groups) {
    const unsigned nm = (unsigned)G.members.size();
    std::vector<const double*> src(nm, nullptr);
    std::vector<double*> dst(nm, nullptr);
    bool any = false;
    for (unsigned k = 0; k < nm; ++k) {
      const int i = G.members[k];
      if (o.status[i] != PFCH_OK) continue;
      src[k] = solution_of(ctx->inst[i], ctx->recs[i]);
      if (!src[k]) return PFCH_E_INTERNAL;
      dst[k] = ctx->inst[i].R[2];
      any = true;
    }
    if (any && (rc = rhs_launch(ctx, G, G.d_members, nm, src, dst))) return rc;
  }
  // error estimates
  std::vector<int> est(n, PFCH_EST_AM3);
  std::vector<double> fac(n, 1.0);
  for (int i = 0; i < n; ++i) {
    Instance& I = ctx->inst[i];
    EstArgs& A = ctx->h_est[i];
    std::memset(&A, 0, sizeof(A));
    A.n = I.npts;
    if (o.status[i] != PFCH_OK) continue;
    A.ut = solution_of(I, ctx->recs[i]);
    if (!A.ut) return PFCH_E_INTERNAL;
    const bool mid = (ad->estimator == PFCH_EST_MIDAB2 ||
                      (ad->estimator == PFCH_EST_AUTO && I.d.scheme == PFCH_MP)) &&
                     I.hist >= 3;
    const double h = dt[i];
    A.f[0] = I.U[I.ucur];
    if (mid) {
      // quadratic through u^n, u^{n-1}, u^{n-2} at t_n + dt~ (eq. fml:midAB2-high-sol)
      const double dn = I.dt_prev, dm = I.dt_nm1;
      est[i] = PFCH_EST_MIDAB2;
      A.f[1] = I.U[1 - I.ucur];
      A.f[2] = I.Um2;
      A.w[0] = (h + dn) * (h + dn + dm) / (dn * (dn + dm));
      A.w[1] = -h * (h + dn + dm) / (dn * dm);
      A.w[2] = h * (h + dn) / (dm * (dn + dm));
      const double rn = 1.0 / 24.0 + 0.125 * (1.0 + dn / h) * (1.0 + 2.0 * dn / h + dm / h);
      fac[i] = 1.0 / (1.0 - 1.0 / (24.0 * rn));
    } else {
      // explicit AM3 value (eq. fml:AM3-high-sol); rho = 0 without history
      const double rho = I.has_prev ? h / I.dt_prev : 0.0;
      A.w[0] = 1.0;
      A.f[3] = I.R[2];
      A.w[3] = h / 6.0 * (3.0 + 2.0 * rho) / (1.0 + rho);
      A.f[4] = I.R[0];
      A.w[4] = h / 6.0 * (3.0 + rho);
      if (I.has_prev) {
        A.f[5] = I.R[1];
        A.w[5] = -h / 6.0 * rho * rho / (1.0 + rho);
      }
    }
  }
  HIPCHK(hipMemcpyAsync(ctx->d_est, ctx->h_est, sizeof(EstArgs) * n, hipMemcpyHostToDevice, ctx->stream));
  {
    const EstArgs* args = ctx->d_est;
    double* part = ctx->d_est_part;
    void* a[] = {&args, &part};
    if ((rc = launch((const void*)&k_adapt_est, dim3(EST_BLOCKS, n), dim3(EST_THREADS), 0, a, ctx->stream)))
      return rc;
  }
  HIPCHK(hipMemcpyAsync(ctx->h_est_part, ctx->d_est_part, sizeof(double) * 2 * EST_BLOCKS * n,
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<double> err(n, INFINITY);
  std::vector<char> take(n, 0);
  int ret = PFCH_OK;
  for (int i = 0; i < n; ++i) {
    if (o.status[i] == PFCH_OK) {
      const double* pp = ctx->h_est_part + (size_t)i * 2 * EST_BLOCKS;
      double se = 0.0, sh = 0.0;
      for (int b = 0; b < EST_BLOCKS; ++b) se += pp[b];
      for (int b = 0; b < EST_BLOCKS; ++b) sh += pp[EST_BLOCKS + b];
      err[i] = sh > 0.0 ? std::sqrt(se / sh) * fac[i] : (se > 0.0 ? INFINITY : 0.0);
    }
    take[i] = o.status[i] == PFCH_OK && (err[i] <= ad->tol || dt[i] <= ad->dt_min);
    if (o.status[i] != PFCH_OK && dt[i] <= ad->dt_min && ret == PFCH_OK) ret = o.status[i];
  }
  const bool want_mass = ctx->stats_detail > 0;
  std::vector<Coef> coefs(n);
  for (int i = 0; i < n; ++i) coefs[i] = coef_of(ctx->inst[i], dt[i]);  // before the history moves
  if ((rc = accept_solutions(ctx, take, dt.data(), o, want_mass, true))) return rc;
  if (want_mass) HIPCHK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < n; ++i) {
    Instance& I = ctx->inst[i];
    if (take[i]) {  // R(u~) becomes R(u^n)
      double* r1 = I.R[1];
      I.R[1] = I.R[0];
      I.R[0] = I.R[2];
      I.R[2] = r1;
    }
    pfch_adapt_result& r = res[i];
    r.dt = dt[i];
    r.err = err[i];
    r.accepted = take[i] ? 1 : 0;
    r.estimator = est[i];
    r.dt_try = next_dt(err[i], ad->tol, dt[i], ad->dt_min, ad->dt_max);
    if ((rc = fill_stats(ctx, o, i, want_mass, take[i], r.solve))) return rc;
  }
  // statistics detail 2: residual of each accepted solution (the accept
  // kept u^n in U[1 - ucur] and u^{n-1} in Um2)
  for (int i = 0; i < n && ctx->stats_detail > 1; ++i) {
    if (!take[i]) continue;
    Instance& I = ctx->inst[i];
    const double* un = I.U[1 - I.ucur];
    if ((rc = residual_norm(ctx, I, I.U[I.ucur], un, coefs[i].c != 0.0 ? I.Um2 : un, coefs[i],
                            &res[i].solve.rnorm_inf)))
      return rc;
  }
  return ret;
}

int pfch_rhs(pfch_ctx* ctx, int32_t inst, const double* v, double* out) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !v || !out || v == out) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  std::vector<const double*> src{v};
  std::vector<double*> dst{out};
  int rc = rhs_launch(ctx, ctx->groups[I.group], I.d_solo, 1, src, dst);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return PFCH_OK;
}

int pfch_rhs_noalloc(pfch_ctx* ctx, int32_t inst, const double* v, double* out) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !v || !out || v == out) return PFCH_E_INVAL;
  Instance& I = ctx->inst[inst];
  if (I.nz > 1) return PFCH_E_UNSUPPORTED;
  const size_t fields = I.d.model == PFCH_FCH ? 3 : 2;
  if (fields * sizeof(c2) * (size_t)I.h.field_stride > SCRATCH_SPECTRAL_BYTES) return PFCH_E_SCRATCH;
  if (!ctx->scratch) return PFCH_E_HIP;
  unsigned char* base = static_cast<unsigned char*>(ctx->scratch);
  const double** slot = reinterpret_cast<const double**>(base);
  {
    void* a[] = {&slot, &v, &out};
    int rc = launch((const void*)&k_rhs_ptrs, dim3(1), dim3(64), 0, a, ctx->stream);
    if (rc) return rc;
  }
  return rhs_kernels(ctx, ctx->groups[I.group], I.d_solo, 1, slot, const_cast<double**>(slot + 1),
                     reinterpret_cast<c2*>(base + SCRATCH_PTR_BYTES));
}

int pfch_solve(pfch_ctx* ctx, int32_t inst, double a, double b, double c, const double* u_n,
               const double* u_nm1, double* x, pfch_stats* st) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size() || !u_n || !x) return PFCH_E_INVAL;
  if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(b) || !std::isfinite(c)) return PFCH_E_INVAL;
  if (c != 0.0 && !u_nm1) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Instance& I = ctx->inst[inst];
  StepSetup ss{};
  ss.un = u_n;
  ss.unm1 = u_nm1 ? u_nm1 : u_n;
  ss.xin = x;
  ss.a = a;
  ss.b = b;
  ss.c = c;
  ss.theta = scheme_mp(I.d.scheme) ? 0.5 : 1.0;
  ss.rho = 0.0;
  int rc;
  if ((rc = launch_setup_solo(ctx, I, ss))) return rc;
  std::vector<int> active{inst};
  if ((rc = run_iterations(ctx, active))) return rc;
  int iters = 0;
  double dn = 0.0;
  const int status = status_of(I, ctx->recs[inst], &iters, &dn);
  if (status == PFCH_OK || status == PFCH_E_NOCONV || status == PFCH_E_NONFINITE) {
    const StopRec& r = ctx->recs[inst];
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
    st->rnorm_inf = NAN;
    st->gain = NAN;
    if ((rc = betas_host(ctx, I, a, st->beta))) return rc;
    if (ctx->stats_detail > 1 && status == PFCH_OK &&
        (rc = residual_norm(ctx, I, x, u_n, u_nm1, Coef{a, b, c, ss.theta}, &st->rnorm_inf)))
      return rc;
  }
  return status;
}


// ---------------------------------------------------------------------------
// Learned initial guess (float32 Fourier neural operator).
// ---------------------------------------------------------------------------

int64_t pfch_fno_num_params(int32_t width, int32_t modes, int32_t layers) {
  if (width < 1 || width > WG_MAXC || modes < 1 || modes > 64 || layers < 1 || layers > 16) return PFCH_E_INVAL;
  return fno_count(width, modes, layers, 2);
}

int64_t pfch_fno_num_params_3d(int32_t width, int32_t modes, int32_t layers) {
  if (width < 1 || width > WG_MAXC || modes < 1 || modes > 64 || layers < 1 || layers > 16) return PFCH_E_INVAL;
  return fno_count(width, modes, layers, 3);
}

void pfch_fno_destroy(pfch_fno* f) {
  if (!f) return;
  (void)hipStreamSynchronize(f->f.s);
  for (void* p : f->f.allocs) (void)hipFree(p);
  for (void* p : f->f.host_allocs) (void)hipHostFree(p);
  for (Resampler* r : f->f.rs) delete r;
  if (f->f.blas) (void)rocblas_destroy_handle(f->f.blas);
  delete f;
}

}  // extern "C"

namespace {

// Network on an Nz x Ny x Nx grid (ndim 3) or an Ny x Nx grid (ndim 2, nz 1).
int fno_create(int ndim, int32_t width, int32_t modes, int32_t layers, int32_t nz, int32_t ny, int32_t nx,
               int32_t max_batch, void* hip_stream, pfch_fno** out) {
  if (!out) return PFCH_E_INVAL;
  *out = nullptr;
  if (pfch_fno_num_params(width, modes, layers) < 0) return PFCH_E_INVAL;
  if (ny < 2 || nx < 2 || nz < 1 || 2 * modes > ny || 2 * modes > nx || max_batch < 1) return PFCH_E_INVAL;
  if (ndim == 3 ? (nz < 2 || 2 * modes > nz) : nz != 1) return PFCH_E_INVAL;
  const long long W = width, M = modes, P = (long long)nz * ny * nx, B = max_batch;
  const long long MM = fno_modes(M, ndim), M2 = 2 * M * M;
  // launch limits of the strided products (batch counts in the grid's z
  // extent) and 32-bit row counts
  if (B * W * nz > 65535 || MM > 65535 || B * W * nz * ny > 0x7fffffffLL || B * W * P > (1LL << 40))
    return PFCH_E_UNSUPPORTED;
  pfch_fno* h = new pfch_fno();
  Fno& F = h->f;
  F.W = width;
  F.M = modes;
  F.L = layers;
  F.ndim = ndim;
  F.nz = nz;
  F.ny = ny;
  F.nx = nx;
  F.maxb = max_batch;
  F.P = P;
  F.MM = MM;
  F.n = fno_count(W, M, layers, ndim);
  F.s = (hipStream_t)hip_stream;
  long long o = 0;
  F.oP = o;
  o += 2 * W;
  F.opb = o;
  o += W;
  for (int l = 0; l < layers; ++l) {
    F.oR.push_back(o);
    o += W * W * MM * 2;
    F.oW.push_back(o);
    o += W * W;
    F.ob.push_back(o);
    o += W;
  }
  F.oQ = o;
  o += W;
  F.oqb = o;
  o += 1;
  auto fail = [&](int rc) {
    pfch_fno_destroy(h);
    return rc;
  };
  auto fal = [&](float** p, long long nfloats) {
    void* q = nullptr;
    const int rc = dalloc(F.allocs, &q, sizeof(float) * (size_t)nfloats);
    *p = (float*)q;
    return rc;
  };
  int rc;
  const long long field = B * W * P;
  if ((rc = fal(&F.theta, F.n)) || (rc = fal(&F.grad, F.n)) || (rc = fal(&F.am, F.n)) || (rc = fal(&F.av, F.n)))
    return fail(rc);
  if ((rc = fal(&F.Fx, 2 * nx * M)) || (rc = fal(&F.Fy, 2 * 2 * M * ny)) || (rc = fal(&F.Gy, 2 * ny * 2 * M)) ||
      (rc = fal(&F.Gx, 2 * M * nx)))
    return fail(rc);
  if (ndim == 3 && ((rc = fal(&F.Fz, 2 * 2 * M * nz)) || (rc = fal(&F.Gz, 2 * nz * 2 * M)) ||
                    (rc = fal(&F.S2, 2 * B * W * nz * M2))))
    return fail(rc);
  F.v.assign(layers + 1, nullptr);
  F.z.assign(layers, nullptr);
  F.vh.assign(layers, nullptr);
  for (int l = 0; l <= layers; ++l)
    if ((rc = fal(&F.v[l], field))) return fail(rc);
  for (int l = 0; l < layers; ++l)
    if ((rc = fal(&F.z[l], field)) || (rc = fal(&F.vh[l], 2 * B * W * MM))) return fail(rc);
  if ((rc = fal(&F.S1, 2 * B * W * nz * ny * M)) || (rc = fal(&F.Yb, 2 * B * W * MM)) ||
      (rc = fal(&F.Yb2, 2 * B * W * MM)))
    return fail(rc);
  if ((rc = fal(&F.xin, B * 2 * P)) || (rc = fal(&F.y, B * P)) || (rc = fal(&F.dy, B * P)) ||
      (rc = fal(&F.dvA, field)) || (rc = fal(&F.dvB, field)))
    return fail(rc);
  F.wg_blocks = (int)std::min<long long>(1024, (B * P + WG_TILE - 1) / WG_TILE);
  // largest (CX + 1) * CY of the three weight-gradient shapes: (W+1)W, 3W, W+1
  if ((rc = fal(&F.wpart, (long long)F.wg_blocks * (W + 2) * W))) return fail(rc);
  if ((rc = fal(&F.lpart, FNO_LOSS_BLOCKS))) return fail(rc);
  {
    void* q = nullptr;
    if ((rc = dalloc(F.allocs, &q, sizeof(double)))) return fail(rc);
    F.loss = (double*)q;
    if ((rc = halloc(F.host_allocs, &q, sizeof(double)))) return fail(rc);
    F.h_loss = (double*)q;
  }
  // DFT matrices, angles reduced exactly in integers before the float64 sin/cos
  {
    const double tp = 2.0 * M_PI;
    std::vector<float> fx(2 * nx * M), gx(2 * M * nx);
    for (long long x = 0; x < nx; ++x)
      for (long long kx = 0; kx < M; ++kx) {
        const double ang = tp * (double)((kx * x) % nx) / nx;
        fx[2 * (x * M + kx)] = (float)std::cos(ang);
        fx[2 * (x * M + kx) + 1] = (float)-std::sin(ang);
        const double c = (kx == 0 || 2 * kx == nx ? 1.0 : 2.0) / (double)P;
        gx[2 * (kx * nx + x)] = (float)(c * std::cos(ang));
        gx[2 * (kx * nx + x) + 1] = (float)(c * std::sin(ang));
      }
    // full axis of length n: forward [2M][n], inverse [n][2M]; row ki >= M
    // holds k = n - 2M + ki
    auto full_axis = [&](long long n, std::vector<float>& fw, std::vector<float>& iv) {
      fw.assign(2 * 2 * M * n, 0.f);
      iv.assign(2 * n * 2 * M, 0.f);
      for (long long ki = 0; ki < 2 * M; ++ki) {
        const long long k = ki < M ? ki : n - 2 * M + ki;
        for (long long y = 0; y < n; ++y) {
          const double ang = tp * (double)((k * y) % n) / n;
          fw[2 * (ki * n + y)] = (float)std::cos(ang);
          fw[2 * (ki * n + y) + 1] = (float)-std::sin(ang);
          iv[2 * (y * 2 * M + ki)] = (float)std::cos(ang);
          iv[2 * (y * 2 * M + ki) + 1] = (float)std::sin(ang);
        }
      }
    };
    std::vector<float> fy, gy, fz, gz;
    full_axis(ny, fy, gy);
    if (ndim == 3) full_axis(nz, fz, gz);
    if (hipMemcpy(F.Fx, fx.data(), fx.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(F.Fy, fy.data(), fy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(F.Gy, gy.data(), gy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(F.Gx, gx.data(), gx.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
        (ndim == 3 && (hipMemcpy(F.Fz, fz.data(), fz.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
                       hipMemcpy(F.Gz, gz.data(), gz.size() * 4, hipMemcpyHostToDevice) != hipSuccess)) ||
        hipMemset(F.theta, 0, sizeof(float) * F.n) != hipSuccess ||
        hipMemset(F.am, 0, sizeof(float) * F.n) != hipSuccess ||
        hipMemset(F.av, 0, sizeof(float) * F.n) != hipSuccess)
      return fail(PFCH_E_HIP);
  }
  *out = h;
  return PFCH_OK;
}

// The resampler between a fine Ny x Nx grid and network F's coarser grid
// (2D), made on first use and owned by the network.  PFCH_E_INVAL unless
// the fine grid is at least the network's on both axes and both are even.
int fno_resampler(Fno& F, int ny, int nx, Resampler** out) {
  *out = nullptr;
  if (F.ndim != 2 || ny < F.ny || nx < F.nx || (ny | nx | F.ny | F.nx) & 1) return PFCH_E_INVAL;
  for (Resampler* r : F.rs)
    if (r->ny == ny && r->nx == nx) {
      *out = r;
      return PFCH_OK;
    }
  if (!F.blas && rocblas_create_handle(&F.blas) != rocblas_status_success) {
    F.blas = nullptr;
    return PFCH_E_HIP;
  }
  Resampler* R = new (std::nothrow) Resampler();
  if (!R) return PFCH_E_NOMEM;
  F.rs.push_back(R);  // freed with the network
  R->ny = ny;
  R->nx = nx;
  R->nb = F.maxb;
  const long long ncy = F.ny, ncx = F.nx, nb = F.maxb;
  auto fal = [&](float** p, long long nfloats) {
    void* q = nullptr;
    const int rc = dalloc(F.allocs, &q, sizeof(float) * (size_t)nfloats);
    *p = (float*)q;
    return rc;
  };
  int rc;
  if ((rc = fal(&R->Dx, nx * ncx)) || (rc = fal(&R->Dy, ncy * ny)) || (rc = fal(&R->Uy, ny * ncy)) ||
      (rc = fal(&R->Ux, ncx * nx)) || (rc = fal(&R->T1, 2LL * nb * ny * ncx)) ||
      (rc = fal(&R->T2, (long long)nb * ny * ncx)) || (rc = fal(&R->Xf, 2LL * nb * ny * nx)) ||
      (rc = fal(&R->yf, (long long)nb * ny * nx)))
    return rc;
  // kernel(n, nc, i, ic) = (1/n) (1 + 2 sum_{k=1}^{nc/2-1} cos 2 pi k (ic/nc - i/n)); the
  // angle's numerator is reduced exactly in integers modulo n nc
  const long double tp = 6.283185307179586476925286766559L;
  auto band = [&](long long n, long long nc, long long i, long long ic) {
    const long long D = n * nc;
    long long d = (ic * n - i * nc) % D;
    if (d < 0) d += D;
    long double acc = 1.0L;
    for (long long k = 1; k < nc / 2; ++k) acc += 2.0L * cosl(tp * (long double)((k * d) % D) / (long double)D);
    return acc;
  };
  std::vector<float> dx(nx * ncx), dy(ncy * ny), uy(ny * ncy), ux(ncx * nx);
  for (long long x = 0; x < nx; ++x)
    for (long long xc = 0; xc < ncx; ++xc) {
      const long double b = band(nx, ncx, x, xc);
      dx[x * ncx + xc] = (float)(b / (long double)nx);
      ux[xc * nx + x] = (float)(b / (long double)ncx);
    }
  for (long long y = 0; y < ny; ++y)
    for (long long yc = 0; yc < ncy; ++yc) {
      const long double b = band(ny, ncy, y, yc);
      dy[yc * ny + y] = (float)(b / (long double)ny);
      uy[y * ncy + yc] = (float)(b / (long double)ncy);
    }
  if (hipMemcpy(R->Dx, dx.data(), dx.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(R->Dy, dy.data(), dy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(R->Uy, uy.data(), uy.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(R->Ux, ux.data(), ux.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
    return PFCH_E_HIP;
  *out = R;
  return PFCH_OK;
}

}  // namespace

extern "C" {

int pfch_fno_create(int32_t width, int32_t modes, int32_t layers, int32_t ny, int32_t nx, int32_t max_batch,
                    void* hip_stream, pfch_fno** out) {
  return fno_create(2, width, modes, layers, 1, ny, nx, max_batch, hip_stream, out);
}

int pfch_fno_create_3d(int32_t width, int32_t modes, int32_t layers, int32_t nz, int32_t ny, int32_t nx,
                       int32_t max_batch, void* hip_stream, pfch_fno** out) {
  return fno_create(3, width, modes, layers, nz, ny, nx, max_batch, hip_stream, out);
}

int pfch_fno_init_params(pfch_fno* f, uint64_t seed) {
  if (!f) return PFCH_E_INVAL;
  Fno& F = f->f;
  std::vector<float> th(F.n, 0.0f);
  uint64_t st = seed;
  auto uni = [&]() {  // splitmix64 -> uniform [-1, 1)
    st += 0x9E3779B97F4A7C15ULL;
    uint64_t z = st;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  };
  const double W = F.W;
  for (long long k = 0; k < 2 * F.W; ++k) th[F.oP + k] = (float)(uni() / std::sqrt(2.0));
  for (int l = 0; l < F.L; ++l) {
    for (long long k = 0; k < (long long)F.W * F.W * F.MM * 2; ++k)
      th[F.oR[l] + k] = (float)((uni() + 1.0) / (2.0 * W * W));
    for (long long k = 0; k < (long long)F.W * F.W; ++k) th[F.oW[l] + k] = (float)(uni() / std::sqrt(W));
  }
  for (long long k = 0; k < F.W; ++k) th[F.oQ + k] = (float)(uni() / std::sqrt(W));
  HIPCHK(hipMemcpyAsync(F.theta, th.data(), sizeof(float) * F.n, hipMemcpyHostToDevice, F.s));
  HIPCHK(hipStreamSynchronize(F.s));
  return PFCH_OK;
}

int pfch_fno_set_params(pfch_fno* f, const float* theta, int64_t n) {
  if (!f || !theta || n != f->f.n) return PFCH_E_INVAL;
  HIPCHK(hipMemcpyAsync(f->f.theta, theta, sizeof(float) * n, hipMemcpyDeviceToDevice, f->f.s));
  return PFCH_OK;
}

int pfch_fno_get_params(pfch_fno* f, float* theta, int64_t n) {
  if (!f || !theta || n != f->f.n) return PFCH_E_INVAL;
  HIPCHK(hipMemcpyAsync(theta, f->f.theta, sizeof(float) * n, hipMemcpyDeviceToDevice, f->f.s));
  HIPCHK(hipStreamSynchronize(f->f.s));
  return PFCH_OK;
}

int pfch_fno_forward(pfch_fno* f, const float* x, float* y, int32_t batch) {
  if (!f || !x || !y || batch < 1 || batch > f->f.maxb) return PFCH_E_INVAL;
  Fno& F = f->f;
  if (fno_forward(F, x, batch, F.s) != hipSuccess) return PFCH_E_HIP;
  HIPCHK(hipMemcpyAsync(y, F.y, sizeof(float) * batch * F.P, hipMemcpyDeviceToDevice, F.s));
  return PFCH_OK;
}

int pfch_fno_grad(pfch_fno* f, const float* x, const float* t, int32_t batch, float* grad, double* loss) {
  if (!f || !x || !t || batch < 1 || batch > f->f.maxb) return PFCH_E_INVAL;
  Fno& F = f->f;
  if (fno_backward(F, x, t, batch, F.s) != hipSuccess) return PFCH_E_HIP;
  if (grad) HIPCHK(hipMemcpyAsync(grad, F.grad, sizeof(float) * F.n, hipMemcpyDeviceToDevice, F.s));
  if (loss) {
    HIPCHK(hipMemcpyAsync(F.h_loss, F.loss, sizeof(double), hipMemcpyDeviceToHost, F.s));
    HIPCHK(hipStreamSynchronize(F.s));
    *loss = *F.h_loss;
  }
  return PFCH_OK;
}

int pfch_fno_adam_step(pfch_fno* f, float lr, float beta1, float beta2, float eps, int32_t step) {
  if (!f || step < 1 || !(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return PFCH_E_INVAL;
  Fno& F = f->f;
  if (step == 1) {
    HIPCHK(hipMemsetAsync(F.am, 0, sizeof(float) * F.n, F.s));
    HIPCHK(hipMemsetAsync(F.av, 0, sizeof(float) * F.n, F.s));
  }
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(F.n)), dim3(256), 0, F.s, F.theta, (const float*)F.grad, F.am, F.av,
                     F.n, lr, beta1, beta2, eps, c1, c2);
  HIPCHK(hipGetLastError());
  return PFCH_OK;
}

int pfch_fno_prepare(pfch_fno* f, const double* u_nm1, const double* u_n, const double* u_np1, double rho,
                     const double norm[4], float* x, float* t) {
  if (!f || !u_nm1 || !u_n || !x || !norm || ((u_np1 == nullptr) != (t == nullptr))) return PFCH_E_INVAL;
  if (!(norm[1] > 0.0) || !(norm[2] > 0.0) || !(norm[3] > 0.0) || !std::isfinite(rho)) return PFCH_E_INVAL;
  Fno& F = f->f;
  hipLaunchKernelGGL(k_fno_inputs, dim3(blocks_for(F.P)), dim3(256), 0, F.s, u_nm1, u_n, u_np1, F.P, rho,
                     norm[0], norm[1], norm[2], norm[3], x, t);
  HIPCHK(hipGetLastError());
  return PFCH_OK;
}

int pfch_fno_prepare_resampled(pfch_fno* f, int32_t ny, int32_t nx, const double* u_nm1, const double* u_n,
                               const double* u_np1, double rho, const double norm[4], float* x, float* t) {
  if (!f || !u_nm1 || !u_n || !x || !norm || ((u_np1 == nullptr) != (t == nullptr))) return PFCH_E_INVAL;
  if (!(norm[1] > 0.0) || !(norm[2] > 0.0) || !(norm[3] > 0.0) || !std::isfinite(rho)) return PFCH_E_INVAL;
  Fno& F = f->f;
  Resampler* R = nullptr;
  int rc = fno_resampler(F, ny, nx, &R);
  if (rc) return rc;
  const long long P = (long long)ny * nx;
  hipLaunchKernelGGL(k_fno_inputs, dim3(blocks_for(P)), dim3(256), 0, F.s, u_nm1, u_n, u_np1, P, rho, norm[0],
                     norm[1], norm[2], norm[3], R->Xf, t ? R->yf : (float*)nullptr);
  HIPCHK(hipGetLastError());
  if (resample_down(F, *R, R->Xf, 2, x, 1, F.s) != hipSuccess) return PFCH_E_HIP;
  if (t && resample_down(F, *R, R->yf, 1, t, 1, F.s) != hipSuccess) return PFCH_E_HIP;
  return PFCH_OK;
}

int pfch_set_fno(pfch_ctx* ctx, int32_t inst, pfch_fno* f, const double norm[4]) {
  if (!ctx || inst < 0 || inst >= (int)ctx->inst.size()) return PFCH_E_INVAL;
  if (int rc_ = drop_spec(ctx)) return rc_;  // instance state or workspaces change
  Instance& I = ctx->inst[inst];
  if (!f) {
    I.fno = nullptr;
    I.fno_rs = nullptr;
    return PFCH_OK;
  }
  if (!norm || !(norm[1] > 0.0) || !(norm[2] > 0.0) || !(norm[3] > 0.0) || !std::isfinite(norm[0]))
    return PFCH_E_INVAL;
  if (I.npts & 1) return PFCH_E_UNSUPPORTED;  // the guess kernels read two points per lane
  int rc;
  Resampler* R = nullptr;
  if (f->f.nz != I.nz || f->f.ny != I.ny || f->f.nx != I.nx) {
    // a network on a coarser grid of the same (2D) rank: its input is the
    // band-limited part of the state sampled on that grid, and its output
    // is interpolated back to the instance's grid
    if (I.nz != 1 || f->f.ndim != 2) return PFCH_E_INVAL;
    if ((rc = fno_resampler(f->f, I.ny, I.nx, &R))) return rc;
  }
  if (!I.xguess) {
    void* q = nullptr;
    if ((rc = dalloc(I.allocs, &q, sizeof(double) * (size_t)I.npts))) return rc;
    I.xguess = (double*)q;
    if ((rc = dalloc(I.allocs, &q, sizeof(double) * (GUESS_BLOCKS + 1)))) return rc;
    I.gpart = (double*)q;
    if ((rc = dalloc(I.allocs, &q, sizeof(double) * (2 + 2 * GUESS_BLOCKS)))) return rc;
    I.gbuf = (double*)q;
    if ((rc = dalloc(I.allocs, &q, sizeof(float) * (size_t)I.npts))) return rc;
    I.gcor = (float*)q;
  }
  I.fno = f;
  I.fno_rs = R;
  for (int k = 0; k < 4; ++k) I.fno_norm[k] = norm[k];
  return reset_gain(ctx, I);
}

}  // extern "C"
