/* mspcg.h -- C interface of the MI355X (gfx950) library for the multisplitting
 * preconditioned conjugate gradient (MSPCG) solve of the even-odd
 * preconditioned Moebius domain-wall-fermion Dirac equation
 * (Tu, "Solving DWF Dirac Equation Using Multisplitting Preconditioned
 * Conjugate Gradient", LATTICE 2018).
 *
 * Conventions shared by every call
 * --------------------------------
 * Lattice: extents L[4] = (Lx, Ly, Lz, Lt), all even; fifth dimension Ls.
 *   lex = x + Lx*(y + Ly*(z + Lz*t)); parity = (x+y+z+t) mod 2 (Sec. 2.2);
 *   cb = lex >> 1 indexes the V/2 sites of one parity.
 * Operator (Sec. 2.2, with the readings of the deferred/garbled formulas):
 *   H psi(x) = sum_mu [(1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)]
 *   chiral basis g_k = [[0,-i s_k],[i s_k,0]], g_t = [[0,1],[1,0]], g5 = diag(1,1,-1,-1)
 *   P_chi = P- S+ + P+ S- with (S+ v)(s) = v(s+1), (S+ v)(Ls-1) = -mf v(0),
 *   (S- v)(s) = v(s-1), (S- v)(0) = -mf v(Ls-1)
 *   M_phi = b + c P_chi,  M_5 = (4-M5) M_phi + 1 - P_chi,  M^4 = -1/2 H M_phi
 *   D_PC = M_5 - M^4_eo M_5^{-1} M^4_oe            (Sec. 2.2, Schur complement)
 *   A    = D_PC^+ D_PC                             (Sec. 2.2, normal equation)
 * Boundary: periodic in space; a hop across the time boundary is multiplied
 *   by t_bc (-1: antiperiodic).  The gauge field passed in is the physical one.
 *
 * Memory
 * ------
 * Gauge: device FP64, [lex][mu][row][col][re,im] (V*4*18 doubles).
 * Fields (mspcg_field): device memory owned by the caller, one parity, in the
 *   storage type `prec`.  A 5D site holds 24 reals, index
 *   k = (spin*3 + colour)*2 + re/im.  They are cut into 16-byte chunks of
 *   C = 2 (F64), 4 (F32) or 8 (F16, BF16) reals, and the fifth dimension is
 *   interleaved inside each chunk position:
 *     real k of site (rhs, cb, s) is element ((((rhs*V/2 + cb)*(24/C) + k/C)*Ls + s)*C + k%C
 *   i.e. [rhs][cb][chunk][s][C]: the Ls spinors of one 4D site are one
 *   contiguous block, and lanes holding consecutive s load consecutive 16-byte
 *   words.  For MSPCG_F16 / MSPCG_BF16 the stored values are v / n with one
 *   FP32 scale n per 5D site in `norm`, laid out [rhs][cb][s]
 *   (n = max |v_i| over the 24 reals; n = 0 means an all-zero site).
 * The library never frees caller memory and keeps no caller pointer after a
 * call returns.  The handle owns its gauge copies, index tables, workspaces
 * and tuned launch shapes.  A handle is not thread-safe: one host thread per
 * handle.
 *
 * Streams and synchronisation
 * ---------------------------
 * Operator calls are asynchronous on `stream` (NULL: the null stream).  The
 * solvers run on the handle's stream and return after synchronising it.
 *
 * Errors
 * ------
 * No call throws.  A negative status means nothing was written to outputs;
 * MSPCG_NOT_CONVERGED means x holds the last iterate and stats are filled.
 * mspcg_last_error() describes the last failure on the calling thread.
 */
#ifndef MSPCG_H
#define MSPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MSPCG_OK = 0,
  MSPCG_NOT_CONVERGED = 1,
  MSPCG_EINVAL = -1,       /* bad argument: odd extent, Ls < 2, parity/precision mismatch, nrhs < 1, NULL */
  MSPCG_EUNSUPPORTED = -2, /* valid but not built: Ls or nrhs above the compiled maximum, halo wrap */
  MSPCG_ENOMEM = -3,       /* device allocation failed */
  MSPCG_EHIP = -4,         /* a HIP runtime call failed */
  MSPCG_ENONFINITE = -5    /* NaN/Inf met in a solver reduction */
} mspcg_status;

typedef enum { MSPCG_F64 = 0, MSPCG_F32 = 1, MSPCG_F16 = 2, MSPCG_BF16 = 3 } mspcg_prec;

/* Largest supported fifth dimension and number of right-hand sides. */
#define MSPCG_MAX_LS 32
#define MSPCG_MAX_NRHS 16

typedef struct {
  int L[4];     /* lattice extents, each even and >= 2 */
  int Ls;       /* fifth dimension, 2 <= Ls <= MSPCG_MAX_LS */
  double M5;    /* domain-wall height */
  double mf;    /* quark mass */
  double b, c;  /* Moebius coefficients (Shamir: b = 1, c = 0); b != 0 */
  int t_bc;     /* -1 antiperiodic, +1 periodic in time */
} mspcg_dwf;

typedef struct {
  void *data;       /* device pointer, layout above */
  float *norm;      /* device pointer [rhs][cb][s], F16/BF16 only (else ignored) */
  mspcg_prec prec;
  int nrhs;         /* 1 <= nrhs <= MSPCG_MAX_NRHS */
  int parity;       /* 0 even, 1 odd */
} mspcg_field;

typedef struct {
  int nblk[4];           /* Dirichlet blocks per dimension (uneven splits allowed) */
  int n_inner;           /* fixed number k of inner CG iterations (>= 0) */
  mspcg_prec inner_prec; /* storage of the inner solve: F32, F16 or BF16 (F64 allowed for tests);
                          * arithmetic is FP32, except that F16 hops form the projected half
                          * spinor in half precision and sum exact half products in FP32 */
  int no_snake;          /* 0 (default): A_s = P_s A P_s with its snake terms (Sec. 2.3);
                          * 1: every hop cut at the block boundary (P_s H P_s), which drops
                          * the snake terms -- the variant Sec. 2.3 argues against, for comparison */
  double inner_tol;      /* 0 (default): exactly n_inner iterations per block (Sec. 3);
                          * > 0: precision-based stopping, the alternative Sec. 3 rejects, for
                          * comparison: a block stops (keeps its iterate) after the first iteration
                          * whose |r_s| <= inner_tol |P_s r|; n_inner is the maximum.  Frozen blocks
                          * still occupy the batched launches, so this changes the preconditioner,
                          * not the cost of an application.  Negative or non-finite: MSPCG_EINVAL */
  int n_sweeps;          /* multisplitting sweeps per application: 0 or 1 (default) is the paper's
                          * single sweep from a zero guess (Sec. 2.4); s > 1 keeps s steps of the
                          * multisplitting iteration (Sec. 2.1), the data of neighbouring blocks
                          * entering through the full residual: z <- z + M (r - A z), with M the
                          * one-sweep preconditioner -- one more FP64 A and one more block solve
                          * per sweep.  Negative: MSPCG_EINVAL */
} mspcg_precond;

typedef struct {
  double tol;            /* stop at true ||b - A x|| / ||b|| <= tol */
  int max_iter;          /* outer iteration limit */
  int reliable_interval; /* replace r by b - A x every this many iterations (0: only at the end) */
  int use_graph;         /* capture the preconditioner in a hipGraph and replay it */
  int timing;            /* 1: fill the time split of mspcg_stats (HIP events around each phase on the
                          * solver's stream; the events add a few microseconds per iteration) */
  int flexible_beta;     /* 0 (default): beta = <z', r'> / <z, r> as Algorithm 1 prints it (Fletcher-Reeves);
                          * 1: beta = <z', r' - r> / <z, r> (Polak-Ribiere), which keeps consecutive search
                          * directions A-conjugate when the preconditioner is not a fixed linear map (a fixed
                          * number of inner CG iterations is not); one more FP64 dot product per iteration */
} mspcg_solver;

typedef struct {
  int outer_iters;          /* iterations of Algorithm 1 */
  long long inner_iters;    /* inner CG iterations summed over outer iterations (per block) */
  double *true_rel_resid;   /* caller-owned host array [nrhs], may be NULL */
  double seconds;           /* wall time of the solve (host clock, includes set-up on first use) */
  double t_outer_op;        /* seconds in the outer operator A = D_PC^+ D_PC (with mspcg_solver.timing) */
  double t_precond;         /* seconds in the preconditioner, local_block_cg (with mspcg_solver.timing) */
  double t_blas;            /* seconds in the outer vector updates and reductions (with mspcg_solver.timing);
                             * all three are 0 when timing is off */
} mspcg_stats;

typedef struct mspcg_handle mspcg_handle;

/* Create a handle for one lattice/action on the current HIP device.  The
 * gauge field (device, FP64, physical links) is copied and repacked on
 * `stream`; the caller may free it after the call returns.
 * MSPCG_EUNSUPPORTED for b = 0 (the hop kernels factor b out of
 * M_phi = b + c P_chi).  Environment read here: MSPCG_AUTOTUNE=0 keeps the
 * default workgroup shapes (no timing of candidates on first use);
 * MSPCG_VERBOSE=n makes the solvers print their residual on stderr every n
 * outer iterations. */
mspcg_status mspcg_create(mspcg_handle **h, const mspcg_dwf *p, const double *gauge_dev_f64, void *stream);
mspcg_status mspcg_destroy(mspcg_handle *h);

/* Hopping block (Sec. 2.2, M^4 = D^w M_phi): `out` has parity p and `in`
 * parity 1-p, same precision and nrhs.  dagger = 0: out = M^4_{p,1-p} in;
 * dagger = 1: out = (M^4_{1-p,p})^+ in. */
mspcg_status dslash_eo(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, int dagger, void *stream);

/* Fifth-dimension block (Sec. 2.2, the constant site-diagonal M_5):
 * out = M_5^{-1} in (dagger = 0) or M_5^{-+} in (dagger = 1), same parity. */
mspcg_status m5inv(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, int dagger, void *stream);

/* Normal operator (Sec. 2.2-2.3): out_e = D_PC^+ D_PC in_e on even sites. */
mspcg_status mdagm(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream);

/* Preconditioner of Sec. 2.4 (M = direct sum of the block operators A_s,
 * each A_s = P_s A P_s with its snake terms, Sec. 2.3): for every block s and
 * right-hand side independently, n_inner textbook CG iterations on
 * A_s z_s = P_s r from z_s = 0 (Sec. 3, fixed inner iterations), then
 * z = sum_s P_s z_s.  r and z are even fields, both F64 or both F32 (F32 is
 * widened to an F64 copy held by the handle and the result narrowed back);
 * other storage types: MSPCG_EUNSUPPORTED.  The inner solve stores its
 * vectors in pc->inner_prec with FP32 arithmetic.  Each right-hand side is
 * scaled to unit RMS before the inner solve (CG_k is scale-equivariant). */
mspcg_status local_block_cg(mspcg_handle *h, mspcg_field *z, const mspcg_field *r, const mspcg_precond *pc,
                            void *stream);

/* One application of the preconditioner's operator: out = (direct sum over
 * blocks s of A_s) in, with A_s = P_s A P_s including its snake terms
 * (Sec. 2.3; pc->no_snake = 1: the truncated variant), computed on the
 * halo-extended block domains with storage pc->inner_prec (FP32 arithmetic
 * unless F64); pc->n_inner is ignored.  in/out: even F64 fields. */
mspcg_status mspcg_block_apply(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, const mspcg_precond *pc,
                               void *stream);

/* Plain CG (Algorithm 1 with M = 1) on A x = b, FP64.  x: initial guess in,
 * solution out.  Each right-hand side has its own alpha and beta. */
mspcg_status cg_solve(mspcg_handle *h, mspcg_field *x, const mspcg_field *b, const mspcg_solver *s,
                      mspcg_stats *st);

/* MSPCG: Algorithm 1 with z = M^{-1} r from local_block_cg, FP64 outer. */
mspcg_status mspcg_solve(mspcg_handle *h, mspcg_field *x, const mspcg_field *b, const mspcg_solver *s,
                         const mspcg_precond *pc, mspcg_stats *st);

/* Source preparation (Sec. 2.2): phihat_e = phi_e - M^4_eo M_5^{-1} phi_o and
 * b = D_PC^+ phihat_e.  phi_e, phi_o, b: F64 fields of parity 0, 1, 0. */
mspcg_status dwf_prepare_rhs(mspcg_handle *h, mspcg_field *b, const mspcg_field *phi_e, const mspcg_field *phi_o,
                             void *stream);

/* Reconstruction: psi_o = M_5^{-1} (phi_o - M^4_oe psi_e).  F64. */
mspcg_status dwf_reconstruct(mspcg_handle *h, mspcg_field *psi_o, const mspcg_field *psi_e,
                             const mspcg_field *phi_o, void *stream);

/* Debug export of the index maps (host arrays, caller-owned):
 * lex_of_cb[V/2] and nbr[V/2][4][2] (neighbour cb, 0 = x+mu, 1 = x-mu) for
 * `parity`; any pointer may be NULL. */
mspcg_status mspcg_debug_site_maps(mspcg_handle *h, int parity, int32_t *lex_of_cb, int32_t *nbr);

/* Debug export of the halo-extended block domains for one blocking: sizes
 * (number of Be / O1 / E2 sites of `block`) and, where non-NULL, their lex
 * indices in the library's order. */
mspcg_status mspcg_debug_block_sites(mspcg_handle *h, const int nblk[4], int block, int32_t counts[3],
                                     int32_t *be_lex, int32_t *o1_lex, int32_t *e2_lex);

/* Measurement: launch one of the four hops of the block operator A_s
 * (Sec. 2.3) for every block at once, `reps` times on `stream`, exactly as an
 * inner CG iteration of local_block_cg launches it (same kernel, domain lists
 * and tuned shape; storage pc->inner_prec, nrhs right-hand sides):
 *   hop 1: B_e -> O1, input M_phi p (stored beside p), M_phi M_5^{-1} epilogue
 *   hop 2: O1 -> E2, plus M_5 applied to the block vector; with the snake
 *          terms also the per-block <p, A_s p> = |D_PC P_s p|^2 partials
 *   hop 3: E2 -> O1, daggered, M_5^{-+} M_phi^+ epilogue
 *   hop 4: O1 -> B_e, daggered, plus M_5^+ y; with the snake terms it
 *          updates the block residual in place, r -= alpha A_s p, with the
 *          |r|^2 partials (repeated launches keep updating r); without them
 *          (pc->no_snake) it forms the <p, A_s p> partials instead
 * on the handle's block work vectors as the last preconditioner call left
 * them (zeros before any).  sites (may be NULL) receives the 4D sites of the
 * launch's input and output domains, summed over blocks (padding excluded):
 * {B_e, O1}, {O1, E2}, {E2, O1}, {O1, B_e} for hops 1..4. */
mspcg_status mspcg_debug_block_hop(mspcg_handle *h, const mspcg_precond *pc, int nrhs, int hop, int reps,
                                   long long sites[2], void *stream);

/* Conversions between storage precisions of one parity (same layout). */
mspcg_status mspcg_convert(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream);

/* Allocation-free variant of mdagm, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops).  Same operator,
 * kernels and layouts as mdagm; the two intermediate fields it needs live in
 * a fixed scratch array of MSPCG_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * first handle created on that GPU until the process ends, instead of
 * handle-owned memory.  Requirements, checked before any device work:
 *   2 * nrhs * (V/2) * Ls * 24 * sizeof(storage real) <= MSPCG_NOALLOC_SCRATCH_BYTES
 *   (plus the F16/BF16 norms, 2 * nrhs * (V/2) * Ls * 4 bytes), else MSPCG_EUNSUPPORTED;
 *   links in the field's precision already prepared by the handle: always for F64 (done by
 *   mspcg_create), for F32/F16/BF16 after any earlier operator call in that precision, else
 *   MSPCG_EUNSUPPORTED.
 * No hipMalloc, hipFree, event creation or launch-shape timing happens in this call: it uses
 * the launch shapes already tuned for this operator on the handle, or the defaults.  Every
 * call on one GPU shares that GPU's scratch array: calls that overlap in time on one GPU (other
 * streams, other threads, other handles) race and give wrong results; serialise them. */
#define MSPCG_NOALLOC_SCRATCH_BYTES (64u << 20)
mspcg_status mdagm_noalloc(mspcg_handle *h, mspcg_field *out, const mspcg_field *in, void *stream);

/* Description of the last error on this thread (empty if none). */
const char *mspcg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MSPCG_H */
