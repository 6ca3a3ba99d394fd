// Host-side declarations shared by the kernel and API translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "../../include/mspcg.h"

namespace mspcg {

// A fifth-dimension operator X = sigma (1 + rho S)(1 - q S)^{-1} per chirality
// (S the chirality's shift of P_chi) is passed to the kernels as its chain
// coefficients [rho, -rho mf, q, sigma, lambda_0 .. lambda_{Ls-1}],
// lambda_i = gamma q^i, gamma = -q mf / (1 + mf q^Ls); the kernels apply it
// as a recurrence along s.
constexpr int kChainHead = 4;

// Epilogues of the hop kernel (what is written for each output 5D site):
enum Epi {
  EPI_SCALE = 0,          // out = scale * hop
  EPI_M5INV = 1,          // out = scale * X hop, X = M_phi M_5^{-1} (undaggered hop) or its transpose (daggered)
  EPI_MPHIDAG = 2,        // out = scale * M_phi^+ hop
  EPI_M5_OTHER = 3,       // out = M_5 other + scale * hop
  EPI_M5DAG_MPHIDAG = 4,  // out = M_5^+ other + scale * M_phi^+ hop
};

// A field [rhs][site][chunk][s][16 bytes] over a list of `stride` sites.
struct Vec {
  void *data = nullptr;
  float *norm = nullptr;  // F16/BF16 only: [rhs][site][s]
  int prec = MSPCG_F64;
  long long stride = 0;   // sites per right-hand side
};

struct HopArgs {
  int nsites;          // output list length
  int Ls, nrhs, nsite_wg;
  const int *site_cb;  // [nsites] cb of the output site in the full lattice (-1: padding)
  const int *nbr;      // [site][8] input index of neighbour d = 2 mu + (0 fwd, 1 bwd); indexed by cb for the
                       // full lattice, by list position for block domains, where a neighbour outside the
                       // domain is stored as -1 - alt (alt: an input index whose data is loaded with weight 0)
  const void *in;
  const float *in_norm;
  long long in_stride;
  void *out;
  float *out_norm;
  long long out_stride;
  const void *links;   // [cb][8][18] for the output parity; sign of the time boundary folded in
  const void *other;   // EPI_M5_OTHER / EPI_M5DAG_MPHIDAG operand
  const float *other_norm;
  long long other_stride;
  const int *other_idx;  // output list position -> index in `other`, -1 outside (zero); nullptr: identity
  double scale;
  const void *mat;     // EPI_M5INV: chain coefficients of X (kChainHead + Ls values in the compute type)
  double mphi_b, mphi_c, mf, m5_alpha, m5_beta;
  double *partial;     // DOT: [gridDim.x][nrhs] partial sums of Re<w, out> (no w: |out|^2)
  // Residual update fused into a block hop (upd_scal set): the value stored
  // is out - alpha * hop result, out read first at the same site (in place),
  // alpha = upd_scal[(upd_blk[site] nrhs + rhs) kScal + 1]; the DOT partials
  // are then |stored value|^2.
  const double *upd_scal;
  const int *upd_blk;
  const void *dotw;
  const float *dotw_norm;
  long long dotw_stride;
};

// Threads of a hop / fifth-dimension workgroup holding nsite_wg sites of nrhs
// right-hand sides (the lane layout depends on Ls); at most 256.
int hop_threads(int Ls, int nrhs, int nsite_wg);
// (site, rhs) groups per 64-lane wave of that layout (0: densely packed lanes)
int hop_groups_per_wave(int Ls, int nrhs);

// Launch the hop kernel for storage `prec`; returns hipSuccess or the launch error.
hipError_t launch_hop(int prec, int dagger, int pre_mphi, int epi, int dot, int global, const HopArgs &a,
                      hipStream_t st);

// out = X in on a site list (identity list), X = a + b P_chi (dag: P_chi^+) or, with inv,
// M_5^{-1} (dag: its transpose) from chain coefficients.
struct Op5Args {
  int nsites, Ls, nrhs, nsite_wg;
  const void *in;
  const float *in_norm;
  void *out;
  float *out_norm;
  long long stride;
  int inv;              // 1: use chain; 0: a + b P_chi
  const void *chain;    // chain coefficients of M_5^{-1} (kChainHead + Ls values in the compute type)
  double a, b, mf;
  int dag;
};
hipError_t launch_op5(int prec, const Op5Args &a, hipStream_t st);

// Precision conversion of [rhs][site][s][24] fields.
hipError_t launch_convert(const Vec &out, const Vec &in, int nrhs, long long nsites5, int Ls, hipStream_t st);

// ------------------------------------------------------------- FP64 BLAS (outer solver)
// n = reals per right-hand side; vectors are [nrhs][n] doubles.
constexpr int kBlasWG = 256;
constexpr int kBlasGrid = 512;  // workgroups per right-hand side (fixed: deterministic sums)
hipError_t blas_dot_partial(const double *a, const double *b, long long n, int nrhs, double *partial, hipStream_t st);
hipError_t blas_reduce(const double *partial, int nparts, int nrhs, double *out, hipStream_t st);
// x += alpha p, r -= alpha q, partial |r|^2; alpha[r] read from scal
hipError_t blas_update_xr(double *x, double *r, const double *p, const double *q, const double *alpha, long long n,
                          int nrhs, double *partial, hipStream_t st);
// p = z + beta p
hipError_t blas_xpay(double *p, const double *z, const double *beta, long long n, int nrhs, hipStream_t st);
// out = a x + b y (host scalars)
hipError_t blas_axpby(double *out, double a, const double *x, double b, const double *y, long long n, int nrhs,
                      hipStream_t st);
// Solver scalars per right-hand side (all device arrays [nrhs]):
//   mode 0: alpha = active ? rho / pap : 0                       (x1 = pap)
//   mode 1: beta = active ? rho_new / rho : 0; rho = rho_new     (x1 = rho_new; Fletcher-Reeves)
//   mode 2: beta = active ? -zq / pap : 0; rho = rho_new         (x1 = rho_new, x2 = <z', A p>, x3 = <p, A p>;
//           Polak-Ribiere, <z', r' - r> / <z, r> with r' - r = -alpha A p)
hipError_t solver_scalars(int mode, int nrhs, const int *active, double *rho, const double *x1, double *out,
                          hipStream_t st, const double *x2 = nullptr, const double *x3 = nullptr);

// ------------------------------------------------------------- block preconditioner
struct BlockArgs {
  int nsites;         // B_e list length (padded)
  int Ls, nrhs, nsite_wg;
  const int *be_cb;   // [nsites]
  const int *be_blk;  // [nsites] block of the site (-1: padding)
  int nblocks;
  const int *be_off;  // [nblocks+1] padded offsets (multiples of the block alignment, itself a multiple of 64)
  double mphi_b, mphi_c, mf;  // M_phi = b + c P_chi (the first block hop reads M_phi p, formed where p is)
};
// r_s = p_s = scale * r(cb), mp_s = M_phi p_s, x_s = 0 (unless xs has no data);
// partial |r_s|^2 per workgroup.
// scale = sqrt(n_total/rr[rhs]).
hipError_t block_gather(int prec, const BlockArgs &b, const Vec &xs, const Vec &rs, const Vec &ps, const Vec &mps,
                        const Vec &rglob, const double *rr, double n_total, double *partial, hipStream_t st);
// z(cb) = v / scale with v = x_s (mode 0), x_s + alpha p_s (mode 1: the last
// inner iteration's x update) or alpha p_s (mode 2: a single inner iteration);
// partial Re<z, r> per workgroup (FP64 r, z; no z data: only the partials)
hipError_t block_scatter(int prec, const BlockArgs &b, const Vec &zglob, const Vec &xs, const Vec &ps,
                         const double *scal, int mode, const Vec &rglob, const double *rr, double n_total,
                         double *partial, hipStream_t st);
// p(cb) = v / scale + beta[rhs] p(cb) (first: p = v / scale), v as in
// block_scatter: the outer direction update with the preconditioned residual
// taken straight from the blocks (FP64 p)
hipError_t block_scatter_xpay(int prec, const BlockArgs &b, const Vec &pglob, const Vec &xs, const Vec &ps,
                              const double *scal, int mode, const double *rr, double n_total, const double *beta,
                              int first, hipStream_t st);
// per (block, rhs): mode 0: alpha = rho/sum(partials) (0 if degenerate)
//                   mode 1: rho_new = sum; beta = rho_new/rho (0 if rho = 0); rho = rho_new
//                   mode 2: rho = sum (initialisation)
hipError_t block_scalars(int mode, const BlockArgs &b, const double *partial, double *scal, hipStream_t st);
// x += alpha p, r -= alpha Ap, partial |r|^2 (the last inner iteration)
hipError_t block_update_xr(int prec, const BlockArgs &b, const Vec &x, const Vec &r, const Vec &p, const Vec &Ap,
                           const double *scal, double *partial, hipStream_t st);
// r -= alpha Ap, partial |r|^2 (the other inner iterations) ...
hipError_t block_update_r(int prec, const BlockArgs &b, const Vec &r, const Vec &Ap, const double *scal,
                          double *partial, hipStream_t st);
// ... then, once beta is known, x += alpha p (first: x = alpha p, x not read),
// p = r + beta p and mp = M_phi p
hipError_t block_update_xp(int prec, const BlockArgs &b, const Vec &x, const Vec &p, const Vec &mp, const Vec &r,
                           const double *scal, int first, hipStream_t st);

// scal layout per (block, rhs): [rho, alpha, beta, pad]
constexpr int kScal = 4;

// Pack the physical FP64 gauge field [lex][mu][3][3] into per-parity site-packed
// links [cb][8][18] (forward U_mu(x), backward U_mu(x-mu)^+, time boundary sign folded).
hipError_t pack_links(int prec, void *out, const double *gauge, const int *lex_of_cb, const int *nbr_lex, int parity,
                      int Vh, int Lt, int Lxyz, double tbc, hipStream_t st);

}  // namespace mspcg
