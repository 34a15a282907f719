// Device-side instance descriptor shared by the kernels and the host runtime.
#pragma once
#include <cstdint>

#include "fft.hpp"

namespace pfch {

enum { MODEL_PFC = 0, MODEL_FCH = 1 };
enum { SCHEME_BDF2 = 0, SCHEME_MP = 1 };
enum { FLAG_PRECOND = 1 };

constexpr uint64_t INF_BITS = 0x7ff0000000000000ull;

// Per-instance stop record, written by the chunk-end kernel.  The host
// mirror also carries the number of the chunk that wrote it: the host uses a
// mirrored record only when that number is the chunk it waited for.
struct StopRec {
  int32_t stop_iter;   // -1 while running; j when ||d_j|| decided the stop;
                       // max_iter when the iteration cap was reached
  int32_t flags;       // FLAG_PRECOND
  uint64_t norm_bits;  // ||d_j||_inf as IEEE bits at the stop
  uint32_t seq;        // host mirror: chunk number of the write (device record: unused)
  int32_t reserved;
};

struct InstDev {
  // geometry (2D: nz = 1)
  int32_t nx, ny, nz, nh;  // nh = nx/2 physical spectral columns
  int32_t model, scheme;
  int32_t rows;            // ny * nz: number of x-rows
  int32_t nparts;          // partial-sum slots written by the setup row kernel
  double kx_scale, ky_scale, kz_scale;  // 2 pi / L per axis
  double inv_p;            // 1 / (nx ny nz)
  // model
  double eps, eta1, eta2, tau, mobility, inv_mobility;
  // solver
  double s, theta_l;
  double lam[8];
  int32_t n_eta, max_iter;
  uint64_t tol_bits;
  // per step (written by the setup kernel, read by the iteration kernels)
  double a, theta, a_over_theta;
  double beta0, beta2;     // averaged-Newton constants (setup column kernel)
  const double* un;        // u^n used by the midpoint blend
  double* acc_dst;         // accept destination of this step (null: the host accepts)
  double* acc_now;         // acc_dst in the chunk whose end stopped the solve, else null
  double* acc_ldst;        // FCH: where the Laplacian of the accepted solution goes
  double* acc_lnow;        // acc_ldst like acc_now
  int32_t lap_hist;        // FCH: this step's set-up took Delta x0 from the kept Laplacians
  int32_t fold_g;          // 2D: no column set-up ran; the step's first column iteration
                           // transforms g and sums the averaged-Newton partials itself
  int32_t resid;           // residual evaluation: the preconditioner is replaced by the
                           // identity, so d_0 = r(x0) = -G'(x0) and norms[0] = ||r(x0)||_inf
  // state buffers
  double* X[3];            // iterate ring x_j at X[j % 3]
  double* DX[3];           // FCH: Laplacian of the iterate, same ring
  double* dun;             // FCH midpoint: Laplacian of u^n
  c2* S;                   // spectral fields [field][tile][rows][4]
  c2* G;                   // setup spectral fields, same layout
  c2* ghat;                // transformed step constant g, tiled like S
  double* part;            // setup partial sums [nparts][2]
  uint64_t* norms;         // ||d_j||_inf bits, [max_iter]
  int32_t* iter_base;      // first iteration index of the current chunk
  int32_t* flags;          // FLAG_* bits raised by kernels
  StopRec* rec;
  StopRec* rec_host;       // pinned host mirror of *rec, written at each chunk end
  const c2* tw_x;          // twiddles for the x length
  const c2* tw_y;          // twiddles for the y length
  const c2* tw_z;          // twiddles for the z length (3D)
  int64_t field_stride;    // rows * nh
  // linear IMEX step: the preconditioner constants are those of the
  // implicit part of the splitting instead of the averaged-Newton means
  int32_t imex;
  double imex_b0, imex_b2;
};

}  // namespace pfch
