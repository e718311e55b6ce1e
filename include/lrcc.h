/*
 * lrcc.h -- C ABI of the MI355X (gfx950) linear-response CCSD library.
 *
 * The library computes frequency-dependent dipole polarizabilities with
 * relativistic (complex, antisymmetrized-spinor) linear-response CCSD,
 * following Chakraborty, Manna, Crawford, Dutta, "A low-cost four-component
 * relativistic coupled cluster linear response theory based on perturbation
 * sensitive natural spinors" (arXiv:2503.23144):
 *   ground state T and energy           Section II.A, Eqs. 9-10
 *   CC Jacobian A                       Eq. 30
 *   Lambda (left) equations             Eqs. 20, 22 (zeroth order)
 *   right response X(w)                 Eqs. 29, 31
 *   left response  Y(w)                 Eqs. 32-34
 *   response function / polarizability  Eq. 35 (alpha = -<<mu_A; mu_B>>)
 *   FNS++ truncated virtual space       Section II.C, Eqs. 41-50
 *
 * Conventions for every call:
 *   - Complex numbers are interleaved {double re, double im}, row-major,
 *     C-contiguous.  Orbital index order: the nocc occupied spinors first,
 *     then the nvir virtual spinors (nmo = nocc + nvir).
 *   - `where` says where a caller buffer lives: LRCC_HOST or LRCC_DEVICE
 *     (a device pointer on the context's GPU).  Input buffers are copied
 *     before the call returns; the caller keeps ownership of everything it
 *     passes in and may free it afterwards.
 *   - Amplitude vectors (T, Lambda, X, Y, sigma in/out) hold the unique
 *     amplitudes: x1[i][a] (nocc*nvir) followed by x2[P(i,j)][P(a,b)] for
 *     i<j, a<b, with the pair index P(p,q) = q(q-1)/2 + p.  Length
 *     lrcc_amplitude_length().  Dot products between left and right
 *     vectors are bilinear (no conjugation) over these unique entries.
 *   - Return value 0 (LRCC_OK) on success, a negative LRCC_E_* code on
 *     failure; lrcc_last_error() then holds a message.  No C++ exception
 *     crosses this interface.  A context is used by one host thread at a
 *     time.  All device work is ordered on the context's HIP stream; calls
 *     that return results to host memory synchronize that stream.
 */
#ifndef LRCC_H
#define LRCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRCC_OK 0
#define LRCC_E_INVALID (-1)   /* null pointer, bad size or option, non-Hermitian input */
#define LRCC_E_STATE (-2)     /* call out of order (e.g. response before ground state) */
#define LRCC_E_NOMEM (-3)     /* device allocation failed */
#define LRCC_E_HIP (-4)       /* HIP runtime error; message has hipGetErrorString */
#define LRCC_E_NOCONV (-5)    /* iteration limit reached; results and stats still written */
#define LRCC_E_SINGULAR (-6)  /* |D_mu -/+ omega| < 1e-8: frequency on a denominator pole */
#define LRCC_E_INTERNAL (-7)

#define LRCC_HOST 0
#define LRCC_DEVICE 1

#define LRCC_FP64 0   /* all arithmetic in complex FP64 */
#define LRCC_MIXED 1  /* Jacobian products in complex FP32 (3M on MFMA), FP64 residuals/updates */

#define LRCC_SIDE_RESIDUAL 0  /* out = Omega(in)                   (Eq. 10)        */
#define LRCC_SIDE_RIGHT 1     /* out = A in + shift * in           (Eqs. 29-30)    */
#define LRCC_SIDE_LEFT 2      /* out = in A + shift * in           (Eqs. 22, 32)   */

#define LRCC_AMP_T 0
#define LRCC_AMP_LAMBDA 1
#define LRCC_AMP_X 2
#define LRCC_AMP_Y 3
#define LRCC_AMP_XMINUS 4  /* X(-w), after lrcc_solve_response_quadratic */

typedef struct lrcc_ctx lrcc_ctx;

typedef struct lrcc_config {
  int device;            /* HIP device ordinal */
  void *stream;          /* hipStream_t to order all work on; NULL = the null stream */
  int precision;         /* LRCC_FP64 or LRCC_MIXED */
  double tol_residual;   /* converged when ||R|| <= tol * ||driving term|| (default 1e-10) */
  int maxit;             /* iteration limit per solve (default 100) */
  int diis_size;         /* DIIS subspace per right-hand side (default 8, 0 = plain Jacobi) */
  int rhs_chunk;         /* right-hand sides per batched Jacobian product (0 = all) */
  int autotune;          /* 1: time the candidate GEMM tiles of each new shape once and keep the
                            fastest (process-wide, per bucket of nearby shapes; cache file from
                            LRCC_AUTOTUNE_CACHE); default 1 */
  int verbose;           /* 0 silent, 1 per-solve summary, 2 per-iteration lines on stderr */
  int graphs;            /* 1: replay the Jacobian-product programs as HIP graphs (captured on the
                            second identical call, replayed from the third); default 1, or 0 when
                            the environment variable LRCC_GRAPHS is "0" */
  int ladder_mode;       /* storage of the vvvv matrix W[P(a,b)][P(e,f)] = <ab||ef> (v^4/4 complex
                            elements per precision) that the ladder contracts with:
                            LRCC_LADDER_FULL (default) the whole matrix;
                            LRCC_LADDER_DIRECT none: every ladder contraction rebuilds W's rows in
                            chunks from the density-fitting factors, (ae|bf) = sum_Q B^Q_ae
                            B^Q_bf, at naux v^4 / 2 extra complex MACs per ladder;
                            LRCC_LADDER_TRIANGLE the upper triangle in row blocks (about half);
                            the lower part is read as conj(W^T), W being Hermitian.
                            Results agree with the full W to rounding. */
  int ladder_mode_fp64;  /* storage of W for the FP64 products of LRCC_MIXED (certification, xi, eta):
                            -1 (default) the same as ladder_mode, else one of the LRCC_LADDER_*
                            values; e.g. FULL FP32 W with a DIRECT FP64 ladder keeps one W in HBM.
                            Ignored with LRCC_FP64 (ladder_mode applies). */
  int memory_mode;       /* LRCC_MEMORY_AUTO (default): LEAN when the RESIDENT footprint of one
                            right-hand side would exceed half the device memory;
                            LRCC_MEMORY_RESIDENT: every integral block dense in HBM;
                            LRCC_MEMORY_LEAN: <ov||vv> only packed over its last pair, and
                            <vv||vo>, <vv||oo> not stored (they equal the conjugates of <ov||vv>
                            and <oo||vv> up to an index order and sign, B being Hermitian); each
                            contraction forms the dense block it reads in chunks of at most 1 GiB.
                            Intermediates only one product reads are freed after it in every mode.
                            Results agree between modes to rounding. */
  int ring_factored;     /* the part of the ring term linear in dt1, t2 . dW(dt1), in the right and
                            left Jacobian products: 1 as dt1 contracted with Z1 = t2 . <ov||vv>-like
                            and Z2 (o v^3 and o^3 v complex elements, formed once per T at o^2 v^4
                            cost), an o^2 v^3 contraction per right-hand side; 0 as the o^3 v^3
                            contraction of t2 with dW per right-hand side; -1 (default) 1 for each
                            executor whose Z1 takes at most 24 GiB at its precision, else 0.
                            Results agree to rounding. */
  int keep_response;     /* 1 (default): the X and Y (or X(w), X(-w)) of every right-hand side stay on
                            the device for lrcc_get_amplitudes; 0: the frequencies are solved in
                            groups (as many as one batched product holds, at least one), alpha of
                            a group is formed before the next group reuses the storage, and only
                            the last group's amplitudes can be read: memory then does not grow
                            with the number of frequencies.  alpha is the same either way. */
} lrcc_config;

#define LRCC_LADDER_FULL 0
#define LRCC_LADDER_DIRECT 1
#define LRCC_LADDER_TRIANGLE 2

#define LRCC_MEMORY_AUTO 0
#define LRCC_MEMORY_RESIDENT 1
#define LRCC_MEMORY_LEAN 2

typedef struct lrcc_stats {
  int iterations;        /* iterations taken */
  int converged;         /* 1 if ||R|| <= tol * ||b|| */
  double residual;       /* final relative residual ||R|| / ||b|| */
  double seconds;        /* wall time of the solve */
  int64_t sigma_evals;   /* Jacobian-vector products (per right-hand side) evaluated */
} lrcc_stats;

/* Fill `cfg` with defaults. */
void lrcc_default_config(lrcc_config *cfg);

/* Create a context on cfg->device.  *ctx is NULL on failure. */
int lrcc_create(lrcc_ctx **ctx, const lrcc_config *cfg);
/* Release every device and host resource of the context (NULL is allowed). */
void lrcc_destroy(lrcc_ctx *ctx);
/* Message of the last failing call on this context ("" if none).  With
   ctx == NULL, the message of the last failing lrcc_create on this thread. */
const char *lrcc_last_error(const lrcc_ctx *ctx);

/* Density-fitting factors B[naux][nmo][nmo] (complex, B^Q Hermitian in pq for
   every Q).  Coulomb integrals (pr|qs) = sum_Q B^Q_pr B^Q_qs; the library
   builds the antisymmetrized blocks <pq||rs> = (pr|qs) - (ps|qr) it needs on
   the device (Section II.B, Eq. 39 uses <ij||ab>) when a later call first
   needs them: here B is copied and checked only, so that a space loaded to
   be truncated (lrcc_fnspp_truncate, lrcc_fns_truncate) forms <oo||vv>
   alone.  An allocation failure of the blocks is reported by that later
   call.  Resets all solutions. */
int lrcc_load_df(lrcc_ctx *ctx, int nocc, int nvir, int naux, const void *B, int where);
/* Fock matrix F[nmo][nmo], Hermitian; may be non-diagonal.  The diagonal
   gives the Jacobi preconditioner D_mu = e_a (+ e_b) - e_i (- e_j). */
int lrcc_load_fock(lrcc_ctx *ctx, const void *F, int where);
/* Dipole (perturbation) matrices mu[ncomp][nmo][nmo], Hermitian, ncomp <= 3. */
int lrcc_load_dipoles(lrcc_ctx *ctx, int ncomp, const void *mu, int where);

/* FNS++ (Section II.C): builds the direction- and frequency-averaged second-
   order vv density (Eqs. 45-50) from MP2 amplitudes, diagonalizes it (Eq.
   41), keeps spinors with |n| > thresh (or the `keep` largest if keep > 0),
   semicanonicalizes (Eqs. 42-44) and rotates B, F and mu of the context into
   the truncated space.  Requires lrcc_load_df, _fock (diagonal) and
   _dipoles.  *nvir_out receives the kept count; occ_out (host, length of the
   original nvir, may be NULL) the occupations sorted by |n| descending. */
int lrcc_fnspp_truncate(lrcc_ctx *ctx, const double *omegas, int nw, double thresh, int keep,
                        int *nvir_out, double *occ_out);
/* Ground-state frozen natural spinors (FNS, Section II.B): the same
   truncation with the MP2 density D_ab = 1/2 sum_ijc t_ij^ac conj t_ij^bc
   (Eq. 40, read as a Hermitian Gram matrix) in place of the perturbed one;
   the baseline FNS++ improves on.  Arguments and results as for
   lrcc_fnspp_truncate (occupations n >= 0 here). */
int lrcc_fns_truncate(lrcc_ctx *ctx, double thresh, int keep, int *nvir_out, double *occ_out);

/* Ground state: solves Omega(t) = 0 from t = 0 (the first Jacobi step gives
   MP2).  ecorr[2] (host) receives the complex correlation energy. */
int lrcc_solve_ground(lrcc_ctx *ctx, double ecorr[2], lrcc_stats *stats);
/* Lambda: solves eta0 + lambda A = 0 at the converged T. */
int lrcc_solve_lambda(lrcc_ctx *ctx, lrcc_stats *stats);
/* Response: for every dipole component B and frequency omegas[k] solves
   (A - w) X = -xi^B and Y (A + w) = -(eta^B + F X^B), batched over all
   right-hand sides, and forms alpha.  per_rhs (host, may be NULL) receives
   2 * ncomp * nw stats: X solves first (k-major, then B), then Y solves. */
int lrcc_solve_response(lrcc_ctx *ctx, int nw, const double *omegas, lrcc_stats *per_rhs);
/* Response by the quadratic route (Eq. 36): for every component B and
   frequency w solves (A - w) X^B(w) = -xi^B and (A + w) X^B(-w) = -xi^B
   (right solves only, batched), then forms
     f_AB(w) = eta^A.X^B(w) + eta^B.X^A(-w) + X^A(-w).F.X^B(w)
   (F, the second derivative of the Lagrangian, applied as one
   Hessian-vector product per X^B(w)) and
   alpha_AB(w) = -1/2 [f_AB(w) + conj f_AB(-w)], read with lrcc_get_alpha.
   It reaches the same alpha as lrcc_solve_response (the two differ by the
   solve residuals), so it serves as an independent check.  per_rhs (host,
   may be NULL) receives 2 * ncomp * nw stats: X(w) solves first, then X(-w).
   Afterwards lrcc_get_amplitudes serves LRCC_AMP_X and LRCC_AMP_XMINUS
   (LRCC_AMP_Y returns LRCC_E_STATE). */
int lrcc_solve_response_quadratic(lrcc_ctx *ctx, int nw, const double *omegas, lrcc_stats *per_rhs);
/* MP2-level correlation energy and polarizability in the current virtual
   space: the terms whose full-space minus truncated-space differences are
   the FNS++ corrections Delta E_MP2 and Delta alpha_MP2 (Eqs. 51-54; call
   once before lrcc_fnspp_truncate and once after, and add the differences to
   the LR-CCSD results of the truncated space).  The paper builds the
   MP2-level response function from the MP2 amplitudes and the perturbed
   amplitudes of Eqs. 46-47; the reading implemented here:
     t(1) = -Omega(0)/D, lambda(1) = -eta0(0)/D (first Jacobi steps of the T
     and Lambda equations; Eq. 39 for a diagonal Fock matrix);
     E_MP2 = E(t(1));
     X^B(+-w) = -xi^B(t(1)) / (Dbar -/+ w) with Dbar the denominators of
     Eqs. 46-47 from the Hbar diagonals of Eqs. 49-50 (orbital energies
     from the Fock diagonal);
     alpha_MP2 from Eq. 36 at (t(1), lambda(1)).
   FP64 throughout.  emp2[2] (host) receives E_MP2; alpha [nw][ncomp][ncomp]
   complex (host or device per `where`).  Needs lrcc_load_df, _fock and
   _dipoles; the context's T and Lambda are kept, X, Y and the alpha of
   lrcc_get_alpha are not touched.  LRCC_E_SINGULAR if a frequency lies on
   an Hbar denominator. */
int lrcc_mp2_response(lrcc_ctx *ctx, int nw, const double *omegas, double emp2[2], void *alpha, int where);
/* alpha[nw][ncomp][ncomp] complex (alpha_AB(w) = -1/2 [f_AB + conj f_BA],
   f_AB = Y^B.xi^A + eta^A.X^B, Eq. 35) from the last lrcc_solve_response. */
int lrcc_get_alpha(lrcc_ctx *ctx, void *alpha, int where);

/* Raw Jacobian products for tests, benchmarks and the autograd wrapper.
   in/out: nvec amplitude vectors; shifts (host, may be NULL = all zero).
   RESIDUAL: out = Omega(in) (nvec must be 1).  RIGHT/LEFT are taken at the
   current T (lrcc_solve_ground or lrcc_set_amplitudes(T) first).
   precision: LRCC_FP64 or LRCC_MIXED (FP32 products).  With where =
   LRCC_DEVICE the call is stream-ordered and does not synchronize; device
   vectors are read and written in place (in == out is allowed and costs a
   copy).  With LRCC_HOST the call returns after out is written. */
int lrcc_sigma(lrcc_ctx *ctx, int side, int nvec, const double *shifts, const void *in, void *out,
               int where, int precision);

/* Length n = nocc*nvir + O*V of one amplitude vector (0 before load_df). */
int64_t lrcc_amplitude_length(const lrcc_ctx *ctx);
/* Checkpoint / resume of T, Lambda, X or Y (idx = k*ncomp + B for X, Y).
   With lrcc_config.keep_response = 0 only the last frequency group's X and Y
   are kept; other idx give LRCC_E_STATE. */
int lrcc_get_amplitudes(lrcc_ctx *ctx, int which, int idx, void *out, int where);
int lrcc_set_amplitudes(lrcc_ctx *ctx, int which, int idx, const void *in, int where);

/* ---- kernel-level entry points (used by the parity tests and the bench) ---- */

/* C = alpha op(A) op(B) + beta C on device buffers, complex, row-major.
   transa/transb: 0 = as stored, 1 = transposed (no conjugation).
   precision LRCC_FP64: 4 real products per complex product on FP64 MFMA;
   LRCC_MIXED: FP32 data, 3 real products (Gauss) on FP32 MFMA, FP32 accumulate.
   alpha, beta: host complex {re, im}.  stream: hipStream_t or NULL.
   Returns LRCC_E_INVALID for a null pointer, a negative size, a leading
   dimension shorter than a row or an unknown precision (message in
   lrcc_last_error(NULL)); asynchronous on `stream` unless the product is
   split over K, in which case it returns after the product is done. */
int lrcc_gemm(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k,
              const double alpha[2], const void *A, int64_t lda, const void *B, int64_t ldb,
              const double beta[2], void *C, int64_t ldc, void *stream);

/* The product of lrcc_gemm, for callers that cannot allocate device memory
   (code under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): it calls no hipMalloc, hipFree or other allocating routine.
   Same arguments, layout and results as lrcc_gemm (the same split over K and
   tile choice; a shape never seen before takes the size heuristic instead of
   being timed).  The split-K partials of deep products live in a static
   device array of 256 MiB per GPU, held from the first call on that GPU until
   the process ends; a product whose partials would not fit returns
   LRCC_E_INVALID (the library caps its splits at that size, so none does
   today).  Fully asynchronous on `stream`.  Every call on one GPU uses the
   same array: calls that overlap in time on one GPU (different streams)
   race on it and must be ordered by the caller. */
int lrcc_gemm_noalloc(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k,
                      const double alpha[2], const void *A, int64_t lda, const void *B, int64_t ldb,
                      const double beta[2], void *C, int64_t ldc, void *stream);

/* Workgroup tile of every later unsplit GEMM launch, process-wide:
   -1 = automatic (the autotuner when a context enables it, else a size
   heuristic; products at most 32 wide take tile 4); 0 = 64 x 64, 1 = 128 x
   64, 2 = 128 x 128 with 4 wavefronts (FP32 only; FP64 runs tile 1), 3 =
   128 x 128 with 8 wavefronts, 4 = 128 x 32.  Every tile computes the same
   product (results agree to rounding); the choice only changes speed.
   Products split over K ignore it.  Returns LRCC_E_INVALID outside -1..4.
   The environment variable LRCC_GEMM_TILE gives the initial value. */
int lrcc_gemm_set_tile(int tile);
/* Tile (0..4 as above) the autotuner chose in this process for the product
   shape (precision LRCC_FP64 or LRCC_MIXED, op(A) m x k, op(B) k x n; ladder
   = 1 for the packed-vvvv ladder contraction of the Jacobian products, which
   runs its own kernel variant), or -1 if that shape has not been timed.  For
   profiles: it names the kernel a trace's or a counter's figures belong to.
   Shapes are timed per bucket (m, n, k above 64 rounded down to their top
   three bits, about 25 % wide), so the answer covers every shape of the
   bucket.  Near-ties (within 2 %) keep the size heuristic's tile. */
int lrcc_gemm_tuned_tile(int precision, int transa, int transb, int64_t m, int64_t n, int64_t k, int ladder);

/* Text of the derived operation lists (host-only, no GPU needed):
   which = 0 residual, 1 right sigma, 2 left sigma, 3 xi, 4 tangent of grad L
   along (X, mu), 5 dE/dt, 6 grad L, 7 F X (tangent of grad L along X),
   8 FNS++ projections of the perturbation over the MP2 doubles, 9 the setup
   of the factored ring terms (Z1, Z2 from t), 10 right and 11 left sigma
   with the factored ring terms (they read Z1 and Z2).
   Writes at most `cap` bytes including the NUL; returns the full length. */
int64_t lrcc_program_text(int which, char *buf, int64_t cap);

/* Time spent in kernels of one class during the last solve or sigma call,
   measured with HIP events on the context's stream (milliseconds, launches).
   cls: 0 = FP32 (3M) packed-vvvv ladder GEMMs, 1 = FP64 (4M) ladder GEMMs,
   2 = all GEMMs.  flops: executed real flops (6 MNK for 3M, 8 MNK for 4M). */
int lrcc_kernel_time(lrcc_ctx *ctx, int cls, double *ms, int64_t *launches, double *flops);
/* Enable (1) or disable (0) the per-launch event timing above.  With graph
   replay on (lrcc_config.graphs), GEMMs inside a replayed graph are not
   timed; the ladder GEMMs are then launched between graph segments so that
   classes 0 and 1 stay complete. */
int lrcc_set_timing(lrcc_ctx *ctx, int on);
/* HIP graphs captured and replayed so far: program runs of the FP64 and
   FP32 executors (lrcc_sigma and the like) and whole solver iterations
   (product, residual, norms, convergence test, DIIS update; the solves run
   each batch's iteration as one graph from its third occurrence).  Either
   pointer may be NULL. */
int lrcc_graph_stats(lrcc_ctx *ctx, int64_t *captures, int64_t *replays);

/* Caller-owned device memory.  lrcc_workspace_bytes estimates (from sizes
   alone, no device needed) the device bytes of the whole pipeline -- load,
   T, Lambda, and X/Y solved in batches of up to nrhs right-hand sides, at
   cfg->precision (cfg may be NULL for the defaults) -- or returns 0 for
   invalid sizes.  FNS++ truncation is not included.  lrcc_set_workspace
   hands the context a device buffer of `bytes` bytes (at least 1 MiB); it
   must come once, right after lrcc_create and before lrcc_load_df
   (LRCC_E_STATE otherwise).  From then on every allocation of the context
   is carved from that buffer and nothing is taken from the device; batch
   sizes adapt to what is free in it, and an allocation that does not fit
   fails with LRCC_E_NOMEM.  The buffer stays owned by the caller, who frees
   it after lrcc_destroy.  lrcc_workspace_peak returns the most of it in use
   at any time so far (0 without a workspace). */
size_t lrcc_workspace_bytes(const lrcc_config *cfg, int nocc, int nvir, int naux, int nrhs);
int lrcc_set_workspace(lrcc_ctx *ctx, void *dptr, size_t bytes);
size_t lrcc_workspace_peak(const lrcc_ctx *ctx);

/* Device memory released by contexts is kept by the library for reuse by
   later allocations in this process (up to half of each device's memory);
   this returns all of it to the devices.  Call it before allocating large
   buffers elsewhere (e.g. with torch).  Synchronizes every device holding
   cached memory. */
int lrcc_trim_memory(void);

/* Build identification string. */
const char *lrcc_build_info(void);

#ifdef __cplusplus
}
#endif
#endif /* LRCC_H */
