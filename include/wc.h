/*
 * wc.h - C interface of libwc, the MI355X (gfx950) Wilson-clover SAP-FGCR library.
 *
 * The method is the mixed-precision Schwarz-preconditioned flexible GCR solver for the
 * Wilson-Dirac operator with clover term of A. Nobile, "Solving the Dirac equation on
 * QPACE" (arXiv:1109.4279): abstract and Sec. 4 (operator, SAP, MR block solver, FGCR,
 * mixed precision by iterative refinement), Sec. 5 (block-contiguous field layout),
 * Sec. 1 (the solves feed the HMC fermion force).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Lattice      dims[4] = (L0, L1, L2, L3), axis 0 = time.  Sites are lexicographic with
 *              x3 fastest.  Every L_mu must be a multiple of the Schwarz block extent b_mu
 *              and L_mu / b_mu must be even (chessboard colouring of the blocks, Sec. 4);
 *              blocks hold at most 256 sites.
 * Operator     D psi(x) = A(x) psi(x) - 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu)
 *                                               + (1 + g_mu) U_mu(x-mu)^dag psi(x-mu)],
 *              A = (4 + m0) + c_sw (i/4) sigma_{mu nu} F_{mu nu}, F the clover-leaf field
 *              strength (Q - Q^dag)/8; chiral gamma basis g0 = [[0,-1],[-1,0]],
 *              gk = [[0,-i s_k],[i s_k,0]], g5 = diag(1,1,-1,-1).
 * Gauge field  complex128 (interleaved re, im) U[4][L0][L1][L2][L3][3][3], row-major 3x3;
 *              U[mu] at x is the link x -> x + mu.
 * Spinors      complex128 psi[nrhs][L0][L1][L2][L3][4][3] (spin, then colour).
 * Pointers     every array argument is a DEVICE pointer on the current HIP device,
 *              owned by the caller, contiguous, at least 16-byte aligned.  The library
 *              copies what it keeps (the links) and never frees caller memory.
 * Streams      `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *              it; only the solver entry points synchronise (once per FGCR restart, to
 *              read the residual norms) and say so.
 * Concurrency  a context owns work fields and a capture stream that its calls reuse: two
 *              calls naming the same context (batched calls included) must not overlap,
 *              whether from two host threads or on two streams without ordering between
 *              them.  Calls on distinct contexts are independent.
 * Errors       every int-returning function returns WC_OK (0) or a negative wc_status;
 *              wc_last_error() gives a message for the calling thread.  Nothing throws
 *              across this interface.  On an error no output has been written unless
 *              the entry point says otherwise.
 */
#ifndef WC_H
#define WC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wc_ctx wc_ctx;

typedef enum {
  WC_OK = 0,
  WC_ERR_ARG = -1,           /* null pointer, nrhs < 1, bad enum or parameter */
  WC_ERR_GEOMETRY = -2,      /* lattice / block shape not allowed (see above) */
  WC_ERR_HIP = -3,           /* HIP runtime error; message kept */
  WC_ERR_OOM = -4,           /* device allocation failed */
  WC_ERR_NOT_CONVERGED = -5, /* solve stopped at maxit or stagnated; x and stats written */
  WC_ERR_BREAKDOWN = -6,     /* NaN/Inf or a vanishing Krylov direction; x and stats written */
  WC_ERR_STATE = -7          /* clover term not created yet */
} wc_status;

/* Storage / arithmetic precision of a kernel.  WC_F16S and WC_BF16S store spinors,
 * links and clover blocks in 16 bits with an FP32 scale per site (per chirality block for
 * the clover) and compute in FP32. */
typedef enum { WC_F64 = 0, WC_F32 = 1, WC_F16S = 2, WC_BF16S = 3 } wc_prec;

typedef enum { WC_FULL = 0, WC_BLOCKS = 1 } wc_region;

typedef struct {
  int nkv;       /* FGCR restart length, 1..32 (Sec. 4: two vectors stored per iteration) */
  int ncy;       /* SAP cycles per preconditioner application, >= 1 */
  int nmr;       /* MR steps per block, >= 1 (Sec. 4: fixed iteration count) */
  int sap_prec;  /* wc_prec of the preconditioner: WC_F64 = plain method, else mixed */
  double tol;    /* stop when ||b - D x|| / ||b|| <= tol, recomputed in FP64 */
  int maxit;     /* cap on FGCR iterations per right-hand side */
  int x0_given;  /* 1: x holds the initial guess (restart point), 0: start from x = 0 */
  int use_graph; /* 1: replay each restart cycle as one captured hipGraph */
  int nr_dirac;  /* right-hand sides per lane in D (0: library / autotuned choice) */
  int nr_sap;    /* right-hand sides per work-group in the block solver (0: library choice) */
  int eo;        /* 1: even/odd-preconditioned block solver (Sec. 4, Table 1), 0: MR on D_Lambda */
  int dagger;    /* 1: solve D^dag x = b, as g5 D^-1 g5 (gamma5-hermiticity of D); 0: D x = b */
  int stag;      /* stagnation test (Sec. 4: restarts): a right-hand side whose FP64 true
                    residual has not dropped over `stag` restarts in a row stops with
                    WC_ERR_NOT_CONVERGED (x and stats written); 0 switches the test off */
  int timing;    /* 1: run the FGCR restart cycles eagerly with HIP events between the
                    phases and report t_sap/t_dirac/t_blas (slower; FGCR only) */
  int basis_prec; /* storage of the FGCR Krylov basis chi_l: WC_F64, or WC_F32 for the
                    single-precision recursion of Sec. 4 (iterative refinement: between
                    restarts D phi_k in FP32 arithmetic, the basis and the recursive
                    residual stored in F32, Gram-Schmidt arithmetic in FP64; the solution
                    and the true residual at every restart in FP64).  FGMRES-DR: WC_F64 only.
                    Errors: WC_ERR_ARG */
  double drop;   /* a restart cycle also ends once its recursive residual is `drop` times
                    the FP64 true residual it started from; 0: none with an FP64 basis,
                    1e-6 with an F32 one (the stored basis bounds how far the recursion
                    can follow the true residual within one cycle); else in (0, 1).
                    FGMRES-DR: 0 only.  Errors: WC_ERR_ARG */
} wc_solver_params;

#define WC_HIST_MAX 64 /* restarts whose true residual wc_solver_stats keeps */

typedef struct {
  int status;          /* wc_status of this right-hand side */
  int iters;           /* FGCR iterations */
  int restarts;        /* restart cycles, each ending in an FP64 true residual */
  int breakdown;       /* 1 if the recursion broke down (NaN/Inf or zero direction) */
  double rel_true_res; /* last FP64 ||b - D x|| / ||b|| */
  double time_ms;      /* solve time of the whole call (same for every rhs of a call) */
  int reorth;          /* FGCR directions that took a second Gram-Schmidt pass */
  int stagnated;       /* 1 if the stagnation test stopped this right-hand side */
  int nhist;           /* entries of res_hist: min(restarts, WC_HIST_MAX) */
  int timed;           /* 1 if the phase times below were measured (params.timing) */
  double t_setup_ms;   /* whole call, stream time: |b|, initial residual */
  double t_cycles_ms;  /* whole call, stream time: the restart cycles */
  double t_finish_ms;  /* reserved (0) */
  double t_sap_ms;     /* with timing: Schwarz preconditioner incl. conversions */
  double t_dirac_ms;   /* with timing: FP64 D (chi = D phi and the true residuals) */
  double t_blas_ms;    /* with timing: Gram-Schmidt, reductions, solution update */
  double res_hist[WC_HIST_MAX]; /* relative FP64 true residual after restart 1, 2, ... */
} wc_solver_stats;

/* Fill p with the library defaults: nkv 16, ncy 5, nmr 4, sap_prec WC_F32, tol 1e-10,
 * maxit 10000, no initial guess, graphs on, automatic RHS tiles, MR block solver, D x = b,
 * stagnation test over 3 restarts, no phase timing, FP64 basis, drop 0. */
void wc_default_params(wc_solver_params* p);

/* Per-context kernel choices (a batched call uses those of its first context).
 * WC_OPT_SAP_CACHE    -1 automatic (default): the block solver keeps the block operator in
 *                     registers when a launch has at most two work items per CU;
 *                     0 reload it in every phase; 1 keep it in registers (FP32-math kernels).
 * WC_OPT_DIRAC_STAGE  -1 automatic (default) and 1: D_w stages each 256-site tile's input
 *                     in LDS (lattices with 256-site blocks, tiles that fit); 0 never.
 * Both select kernels only; results agree to rounding.  Errors: WC_ERR_ARG. */
typedef enum { WC_OPT_SAP_CACHE = 0, WC_OPT_DIRAC_STAGE = 1 } wc_option;
int wc_set_option(wc_ctx* ctx, int option, int value);

/* Right-hand sides handled together, per storage precision prec: nr_dirac per lane of D
 * (1..4), nr_sap per work-group of the plain block solver and nr_sap_eo of the even/odd one
 * (1..2; FP64 1).  0 leaves the library's choice (or the autotuner's).  Errors: WC_ERR_ARG. */
int wc_set_tiles(wc_ctx* ctx, int prec, int nr_dirac, int nr_sap, int nr_sap_eo);

/* Create a context for one lattice: copies the gauge field U (device, complex128, see
 * above) and lays it out block-major with Schwarz blocks block[4] (Sec. 5: points of one
 * block are contiguous).  bc_t = +1 periodic, -1 antiperiodic fermions in time.
 * Errors: WC_ERR_ARG (null), WC_ERR_GEOMETRY (dims/block), WC_ERR_OOM, WC_ERR_HIP. */
int wc_create_gauge(wc_ctx** ctx, const int dims[4], const int block[4], const void* U, int bc_t, void* stream);

/* Build the clover blocks A_+-(x) from the links: (4 + m0) + c_sw (i/4) sigma F (abstract,
 * Sec. 4; two 6x6 Hermitian chiral blocks per site).  Replaces any previous clover. */
int wc_create_clover(wc_ctx* ctx, double m0, double csw, void* stream);

/* Re-lay the context out for another Schwarz block shape (used by the autotuner). */
int wc_set_block(wc_ctx* ctx, const int block[4], void* stream);

/* Copy the clover blocks out: A[V][2][6][6] complex128 (lexicographic sites; block 0 acts
 * on spins 0,1, block 1 on spins 2,3; row index 3*spin + colour), Hermitian-completed. */
int wc_clover_export(wc_ctx* ctx, void* A, void* stream);

/* out = D in (region WC_FULL) or the block-diagonal sum of the Dirichlet block operators
 * D_Lambda in (WC_BLOCKS: hops between different blocks dropped, Sec. 4).  dagger = 1
 * applies D^dag = g5 D g5.  prec selects storage/arithmetic; inputs and outputs are
 * complex128 in any case (converted on the device).  in and out must not overlap. */
int wc_apply_D(wc_ctx* ctx, void* out, const void* in, int nrhs, int prec, int region, int dagger, void* stream);

/* One Schwarz half-sweep (Sec. 4): nmr MR steps from a zero start on every block of the
 * given colour, source rho.  On return z holds the block solutions on that colour and 0
 * elsewhere; rho holds the block residual rho - D_Lambda z on that colour and 0 elsewhere.
 * eo = 0: MR on the Dirichlet block operator D_Lambda.  eo = 1: the even/odd-preconditioned
 * block solver (Sec. 4, Table 1): with the block's sites split by parity (sum of the
 * coordinates mod 2) and H the in-block hops, MR on S = A_ee - H_eo A_oo^-1 H_oe for the
 * even half, source eta_e - H_eo A_oo^-1 eta_o; then z_o = A_oo^-1 (eta_o - H_oe z_e).  The
 * block residual is then zero on the odd sites.  The first eo call on a context builds
 * A^-1 on the odd sites (FP64 Gauss-Jordan, then the storage precision). */
int wc_sap_block_mr(wc_ctx* ctx, void* z, void* rho, int nrhs, int colour, int nmr, int prec, int eo, void* stream);

/* psi = M_SAP eta: ncy cycles of the Schwarz alternating procedure from psi = 0 (Sec. 4):
 * white blocks, residual update on their neighbours' borders, black blocks, update.
 * eo selects the block solver as for wc_sap_block_mr. */
int wc_sap(wc_ctx* ctx, void* psi, const void* eta, int nrhs, int ncy, int nmr, int prec, int eo, void* stream);

/* Solve D x = b (D^dag x = b when p->dagger) for nrhs right-hand sides with
 * SAP-preconditioned restarted FGCR (Sec. 4).
 * The preconditioner runs in p->sap_prec; chi = D phi, Gram-Schmidt, the residual update,
 * the solution update and the true residual stay in FP64.  st (may be NULL) receives nrhs
 * entries.  Synchronises `stream` once per restart.  A right-hand side with b = 0 returns
 * x = 0 after zero iterations, also when an initial guess was given.  Returns WC_OK when
 * every rhs converged, else the first failing status (x is written regardless). */
int wc_fgcr_solve(wc_ctx* ctx, void* x, const void* b, int nrhs, const wc_solver_params* p, wc_solver_stats* st,
                  void* stream);

/* Solve D x = b with SAP-preconditioned FGMRES-DR (Sec. 4): flexible GMRES cycles of
 * p->nkv Arnoldi steps (FP64 basis, classical Gram-Schmidt; preconditioner as for
 * wc_fgcr_solve); at a restart the kdefl harmonic Ritz vectors of the cycle's matrix Hbar
 * with the smallest |theta| (wc_harmonic_ritz), orthonormalised and augmented with the
 * least-squares residual, start the next cycle, which then adds nkv - kdefl steps.
 * kdefl = 0 is restarted FGMRES.  0 <= kdefl < nkv.  The least squares, the harmonic Ritz
 * pairs and the deflation basis are computed on the host in FP64 at every restart (the
 * host synchronises `stream` twice per restart); the Arnoldi cycle runs on the device (one
 * captured hipGraph per first column when p->use_graph).  The basis is orthogonalised by
 * classical Gram-Schmidt applied twice, since it is carried over restarts.  If any
 * unconverged rhs ended its cycle with fewer than kdefl + 1 columns, its recomputed FP64
 * residual exceeds 10x the cycle's least-squares residual, or the small problem is
 * singular, that restart is taken without deflation, from the true residual.  Stats and errors as wc_fgcr_solve; iters counts Arnoldi
 * steps (preconditioner applications). */
int wc_fgmres_dr_solve(wc_ctx* ctx, void* x, const void* b, int nrhs, const wc_solver_params* p, int kdefl,
                       wc_solver_stats* st, void* stream);

/* The same for nlat lattices of different sizes solved together: every kernel of the
 * solve is one launch over all lattices and right-hand sides (the block solver one per
 * block volume among them).  x[i], b[i] are the lattice-i arrays with nrhs[i] right-hand
 * sides; st receives sum(nrhs) entries.  The work fields and captured cycles of a list of
 * lattices and rhs counts are kept for the next call with the same list (device memory of
 * about (2 nkv + 6) FP64 fields of sum(nrhs) right-hand sides), until one of its contexts
 * changes its block layout or is destroyed; such a call counts as a call on every one of
 * its contexts for the concurrency rule above. */
int wc_fgcr_solve_batch(wc_ctx* const* ctxs, int nlat, void* const* x, const void* const* b, const int* nrhs,
                        const wc_solver_params* p, wc_solver_stats* st, void* stream);

/* FGMRES-DR (as wc_fgmres_dr_solve) for nlat lattices of different sizes solved together,
 * arguments as wc_fgcr_solve_batch. */
int wc_fgmres_dr_solve_batch(wc_ctx* const* ctxs, int nlat, void* const* x, const void* const* b, const int* nrhs,
                             const wc_solver_params* p, int kdefl, wc_solver_stats* st, void* stream);

/* G = coef * dL/dU for L = sum_r Re <Y_r, D X_r> in torch's complex-gradient convention
 * (dL = Re sum tr(G^dag dU)), complex128 [4][L0..L3][3][3].  Hopping and clover terms
 * (product rule over the plaquette leaves).  Used for the backward of D and of D^-1. */
int wc_link_grad(wc_ctx* ctx, void* G, const void* Y, const void* X, int nrhs, double coef, void* stream);

/* The pseudofermion action S = phi^dag (D^dag D)^-1 phi = ||Y||^2 (Sec. 1: the HMC action of
 * the fermion determinant): Y = D^-dag phi and X = D^-1 Y by two solves with p (complex128
 * spinors, caller-owned, written), *S (host) = ||Y||^2 summed on the device in FP64.  st
 * (may be NULL) gets 2 entries.  Errors as wc_fgcr_solve; Y, X, S are written regardless. */
int wc_pseudofermion_action(wc_ctx* ctx, const void* phi, const wc_solver_params* p, double* S, void* Y, void* X,
                            wc_solver_stats* st, void* stream);

/* out = coef * in for nrhs complex128 spinor fields of the context's lattice (the action's
 * derivative with respect to phi is 2 X).  out may equal in. */
int wc_spinor_scale(wc_ctx* ctx, void* out, const void* in, int nrhs, double coef, void* stream);

/* wc_apply_D without any device allocation, for callers that cannot allocate: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * layouts and results are those of wc_apply_D (same kernels, bit-identical output).  The
 * packed input and output fields and the kernels' work list live in a fixed scratch array
 * of 128 MiB per GPU that the library holds until the process ends; a call needs
 * 256 B + 16 B per 256-site chunk and rhs tile + 2 x nrhs x V x (192 B FP64, 96 B FP32,
 * 52 B 16-bit), e.g. 16^3 x 32 in FP64 up to 2 right-hand sides.  Larger requests return
 * WC_ERR_ARG.  The operator must already be resident in prec (the FP64 one always is; any
 * earlier wc_apply_D or solve in prec makes it so), else WC_ERR_STATE.  Every call on a GPU
 * shares that GPU's scratch array, so calls that overlap on one GPU (other streams, other
 * host threads, other contexts) race; nothing in the array needs clearing between calls. */
int wc_apply_D_noalloc(wc_ctx* ctx, void* out, const void* in, int nrhs, int prec, int region, int dagger,
                       void* stream);

/* Harmonic Ritz pairs of an Arnoldi cycle (Sec. 4, the deflated restarts of FGMRES-DR),
 * computed on the host in FP64: eigenpairs of H + |h_{m+1,m}|^2 H^-H e_m e_m^T with H the
 * top m x m block of the (m+1) x m matrix Hbar.  Hbar: host complex128, column-major with
 * leading dimension m+1.  theta (m complex128) and G (m x m complex128, column-major,
 * unit columns) receive the pairs sorted by increasing |theta|.  1 <= m <= 32.
 * Errors: WC_ERR_ARG, WC_ERR_BREAKDOWN (H singular or no convergence). */
int wc_harmonic_ritz(int m, const void* Hbar, void* theta, void* G);

/* Pseudofermion force of S = phi^dag (D^dag D)^-1 phi (Sec. 1: the HMC force from the
 * fermion determinant): Y = D^-dag phi and X = D^-1 Y by two solves with p, then
 * F_mu(x) = sum_a (dS/d eps_a) T^a for U_mu(x) -> exp(eps_a T^a) U_mu(x), T^a = i lambda_a / 2,
 * a traceless anti-Hermitian complex128 [4][L0..L3][3][3].  Y, X may be NULL or receive
 * the two solutions (complex128 spinors).  st (may be NULL) gets 2 entries. */
int wc_force(wc_ctx* ctx, void* F, const void* phi, const wc_solver_params* p, wc_solver_stats* st, void* Y,
             void* X, void* stream);

/* Autotune for solves of nrhs right-hand sides whose preconditioner runs in prec: time the
 * RHS tile of D in prec, of the outer solver's FP64 D (and, for 16-bit prec, its FP32 D of
 * an F32 basis) and of both block solvers in prec, and keep the fastest in the context.
 * nr_out[0..3] receive the chosen tiles: D in prec, FP64 D, plain block solver, even/odd
 * block solver. */
int wc_autotune(wc_ctx* ctx, int nrhs, int prec, int nr_out[4], void* stream);

/* Choose the Schwarz block shape of the context among the valid shapes with at most 256
 * sites by timing a short solve (tolerance p->tol) of one Gaussian source for each;
 * re-lays the context out for the fastest.  block_out receives it. */
int wc_autotune_block(wc_ctx* ctx, const wc_solver_params* p, int block_out[4], void* stream);

/* Timing helpers for the benchmark: run the D kernel (or one Schwarz half-sweep) iters
 * times back to back on internal fields between two HIP events on `stream`; *ms gets the
 * mean time per launch.  Synchronises `stream`. */
int wc_bench_dirac(wc_ctx* ctx, int prec, int nrhs, int region, int iters, double* ms, void* stream);
int wc_bench_sap(wc_ctx* ctx, int prec, int nrhs, int nmr, int eo, int iters, double* ms, void* stream);

/* Release everything the context owns. */
void wc_destroy(wc_ctx* ctx);

/* Message of the last error on this thread (static storage, valid until the next call). */
const char* wc_last_error(void);

/* Interface version: 100 * major + minor (2.1). */
int wc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WC_H */
