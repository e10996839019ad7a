/*
 * libdd: two-level DD-alpha-AMG for the Wilson-clover operator on one AMD
 * Instinct gfx950 GPU.  C ABI: plain pointers and sizes, no C++ types.
 *
 * The method is the one of Ishikawa & Kanamori, "Porting DDalphaAMG solver to
 * K computer" (LATTICE2018), Sec. 2: adaptive test vectors, aggregation with
 * chirality split (Eq. 1), Galerkin coarse operator (Eq. 2), restriction and
 * prolongation (Eqs. 3-4), the preconditioner M (Eq. 5) with SAP post-smoothing
 * and an even-odd coarse GMRES, inside a flexible GMRES outer solver.  The
 * problem solved is D x = b for given links, mass m0 (kappa = 1/(8 + 2 m0)) and
 * c_sw (Sec. 1), as a batch of right-hand sides per gauge field (Sec. 4).
 *
 * Conventions shared with the canonical host layouts
 *   site     = x + Lx*(y + Ly*(z + Lz*t)); directions mu = 0..3 <-> x, y, z, t
 *   links    : complex128 [V][4][3][3]        (site, mu, row, column)
 *   fine vec : complex128 [nrhs][V][4][3]     (rhs, site, spin, colour)
 *   coarse   : complex128 [nrhs][Vc][2][n]    (rhs, coarse site, chirality, vector)
 *              coarse site = lexicographic index of the block coordinates
 *   gamma matrices in the chiral representation, gamma5 = diag(1,1,-1,-1)
 *   D psi(x) = A(x) psi(x) - 1/2 sum_mu [(1-g_mu) U_mu(x) psi(x+mu)
 *                                        + (1+g_mu) U_mu(x-mu)^dag psi(x-mu)]
 *   A(x) = (4 + m0) - (c_sw/32) sum_{mu,nu} g_mu g_nu (x) (Q_mu,nu(x) - Q_nu,mu(x))
 *   hops that wrap around in t are multiplied by bc_t.
 *
 * Internal ("packed") vectors are the device layouts the kernels use; they are
 * reached only through dd_pack_* / dd_unpack_* and sized by dd_*_vec_bytes.
 *
 * Ownership: the library owns every handle and its own device workspace, which
 * counts against the context's HBM budget.  Callers own every vector buffer
 * they pass (device pointers).  Threads may share a dd_ctx (its allocation
 * accounting is locked), each driving its own dd_gauge / dd_mg / dd_solve_state
 * on its own stream; one handle is used by one thread at a time.  Apply calls
 * are asynchronous on `stream` (a hipStream_t, NULL = default stream).
 * dd_setup and the solve calls synchronise `stream` at their convergence checks.
 *
 * Errors: every call returns a dd_status; nothing aborts or throws across the
 * ABI.  dd_last_error() gives the text of the last error that the calling
 * thread met on a context ("" if none).
 */
#ifndef DD_H
#define DD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DD_OK = 0,
  DD_EINVAL = 1,   /* bad argument (null pointer, unknown dtype, nrhs < 1, ...) */
  DD_ESHAPE = 2,   /* lattice / block / n_vec combination not supported          */
  DD_ENOMEM = 3,   /* device allocation failed                                   */
  DD_EBUDGET = 4,  /* the request would exceed the context's HBM budget          */
  DD_ENOCONV = 5,  /* solver stopped at max_outer_iters; x holds the best iterate */
  DD_ENAN = 6,     /* non-finite right-hand side or breakdown                    */
  DD_EDEVICE = 7,  /* HIP runtime error                                          */
  DD_ESTATE = 8    /* object in use (e.g. gauge referenced by a multigrid)       */
} dd_status;

/* Arithmetic / storage type of an operation.  DD_F64: FP64 vectors and
 * operands.  DD_F32: FP32 vectors and operands.  DD_F16 / DD_BF16: FP32
 * vectors and arithmetic with links, clover, clover inverse and test vectors
 * stored in half / bfloat16 (round to nearest even from FP32). */
typedef enum { DD_F64 = 0, DD_F32 = 1, DD_F16 = 2, DD_BF16 = 3 } dd_dtype;

typedef struct dd_ctx dd_ctx;
typedef struct dd_gauge dd_gauge;
typedef struct dd_mg dd_mg;

/* The discretised problem.  `block` is the domain tiling (the paper's 4^4
 * blocks, Sec. 4): each block is one coarse site and one SAP domain.  Every
 * block edge must be a power of two >= 2, divide L, and leave an even number
 * of blocks in every direction (red-black SAP and coarse even-odd need it). */
typedef struct {
  int32_t L[4];
  int32_t block[4];
  int32_t bc_t;      /* -1 antiperiodic, +1 periodic in t */
  double m0;         /* mass; kappa = 1/(8 + 2 m0) */
  double c_sw;
} dd_problem;

/* Multigrid parameters (defaults from dd_mg_params_default follow the paper:
 * Sec. 2 four setup iterations, coarse stop at 5e-2; Sec. 4 N_SAP = 4). */
typedef struct {
  int32_t agg_block[4];       /* must equal the gauge's block                     */
  int32_t sap_block[4];       /* must equal the gauge's block                     */
  int32_t n_vec;              /* test vectors n (even, Sec. 3), 2n coarse dof     */
  int32_t setup_iters;        /* adaptive iterations after the initial solves     */
  int32_t init_sap_apps;      /* SAP approximate solves on the random vectors     */
  int32_t sap_sweeps;         /* nu: SAP sweeps per smoother application          */
  int32_t sap_mr_iters;       /* fixed MR iterations per domain solve             */
  int32_t coarse_restart;     /* coarse GMRES restart length                      */
  int32_t coarse_max_iters;   /* coarse GMRES iteration cap                       */
  int32_t coarse_fixed_iters; /* > 0: exactly this many coarse iterations         */
  int32_t fgmres_restart;     /* outer FGMRES(m)                                  */
  int32_t max_outer_iters;
  double coarse_tol;          /* relative residual of the coarse Schur system    */
  dd_dtype inner_dtype;       /* DD_F64: all-FP64 preconditioner; else FP32      */
  dd_dtype store_dtype;       /* operand storage inside M (F64/F32/F16/BF16)      */
  uint64_t seed;              /* random starting vectors of dd_setup              */
  int32_t coarse_cgs_passes;  /* classical Gram-Schmidt passes in the coarse GMRES (1 or 2) */
  int32_t outer_cgs_passes;   /* classical Gram-Schmidt passes in the FP64 outer FGMRES (1 or 2; default 2) */
} dd_mg_params;

typedef struct {
  /* coarse_iters_total: Arnoldi steps of the coarse even-odd GMRES summed over the call's V-cycles
   * (with a third level: steps of the level-2 FGMRES cycles) */
  int32_t outer_iters, restarts, coarse_iters_total, converged;
  double true_relres;          /* |b - D x| / |b| with the FP64 operator */
  double t_setup_s, t_solve_s;
  /* algorithmic HBM bytes and flops of the whole call (all right-hand sides):
   * the sum over its instrumented kernel launches of each launch's model
   * (operands and vectors read once, outputs written once; useful flops) */
  int64_t bytes_model, flops_model;
} dd_solve_info;

/* ---- context -------------------------------------------------------------- */
dd_status dd_ctx_create(int device, size_t hbm_budget_bytes, dd_ctx** out);
void dd_ctx_destroy(dd_ctx* ctx);
const char* dd_status_str(dd_status s);
const char* dd_last_error(const dd_ctx* ctx);
size_t dd_ctx_bytes_in_use(const dd_ctx* ctx);
void dd_mg_params_default(dd_mg_params* p);

/* Launch shapes and coarse storage.  The first three give bit-identical results
 * for every choice (see dd_autotune).  coarse_half, coarse_basis_half and
 * coarse_mfma_half change the rounding of the coarse-level arithmetic, which
 * only the FGMRES outer iteration count can see (the outer solver is flexible,
 * Sec. 2). */
typedef struct {
  int32_t sap_wpe;        /* SAP waves per SIMD the registers allow: 2 or 3          */
  int32_t dirac_threads;  /* D apply workgroup size, 64, 128 or 256 (blocks other than 4^4; 4^4 blocks
                             take one 256-thread workgroup per block)                */
  int32_t coarse_spw;     /* coarse apply: target waves per workgroup, 2, 4 or 8 (sites per workgroup =
                             max(1, coarse_spw / ceil(2n / 16)), at most 4)          */
  int32_t coarse_half;    /* half-precision setups: coarse blocks in FP16/BF16 (1) or FP32 (0);
                             never changed by dd_autotune */
  int32_t coarse_basis_half; /* FP32 coarse GMRES: Krylov basis stored in FP16 (1) or FP32 (0);
                                never changed by dd_autotune */
  int32_t coarse_mfma_half;  /* with half-precision coarse blocks (coarse_half = 1): multiply them on
                                FP16 / BF16 matrix cores with x rounded to the same type and FP32
                                accumulation (1), or convert them to FP32 (0); never changed by
                                dd_autotune */
  int32_t sap_dom_rhs;       /* SAP on 4^4 domains with FP16 / BF16 operands: one workgroup per domain,
                                its operator staged in LDS once and shared by the right-hand sides,
                                taken 2 at a time (links and inverse in LDS, two workgroups per CU) or
                                4 at a time (clover in LDS too, one per CU); 0 = one workgroup per
                                (domain, RHS) in layout sap_wpe.  Same arithmetic, rounding may differ
                                in the last place. */
  int32_t sap_persist;       /* with sap_dom_rhs > 0: every sweep and colour of a smoother application in
                                one cooperative launch whose workgroups (as many as the CUs hold) meet
                                at a grid barrier between colours (1), or one launch per colour (0).
                                Same bits.  Work captured into a graph always takes the launch form. */
} dd_tuning;

/* ---- gauge field (field preparation) ---------------------------------------
 * Copies the links (host, canonical complex128), builds the clover term from
 * the four plaquette leaves of every plane and inverts its two Hermitian 6x6
 * chirality blocks in FP64 (Sec. 3 stores the full inverse, packed as 6 real
 * plus 15 complex numbers per block).  Keeps FP64 copies for the outer
 * operator and lazily makes the storage-dtype copies the inner solvers use.
 * The caller may free links_host on return. */
dd_status dd_gauge_create(dd_ctx* ctx, const dd_problem* prob, const double* links_host,
                          dd_gauge** out);
dd_status dd_gauge_destroy(dd_gauge* g);   /* DD_ESTATE while a dd_mg references it */
/* New bare mass m0 (kappa = 1/(8 + 2 m0)) on the same links: rebuilds the
 * clover term and its inverse and refreshes the storage copies.  DD_ESTATE
 * while a dd_mg references g (use dd_setup_update_mass), DD_EINVAL for a
 * non-finite m0. */
dd_status dd_gauge_set_mass(dd_gauge* g, double m0);

/* ---- vectors ------------------------------------------------------------------ */
size_t dd_fine_vec_bytes(const dd_gauge* g, dd_dtype dt, int nrhs);
size_t dd_coarse_vec_bytes(const dd_mg* mg, dd_dtype dt, int nrhs);
/* canonical complex128 device buffer <-> packed device buffer of dtype dt */
dd_status dd_pack_fine(const dd_gauge* g, dd_dtype dt, int nrhs, const double* canon_dev,
                       void* packed_dev, void* stream);
dd_status dd_unpack_fine(const dd_gauge* g, dd_dtype dt, int nrhs, const void* packed_dev,
                         double* canon_dev, void* stream);
dd_status dd_pack_coarse(const dd_mg* mg, dd_dtype dt, int nrhs, const double* canon_dev,
                         void* packed_dev, void* stream);
dd_status dd_unpack_coarse(const dd_mg* mg, dd_dtype dt, int nrhs, const void* packed_dev,
                           double* canon_dev, void* stream);

/* ---- fine operator and smoother ---------------------------------------------------
 * dd_dirac_apply: out = D in for nrhs packed vectors (Sec. 3: hopping term and
 * clover term).  DD_F64 uses the FP64 operands; DD_F32/F16/BF16 use the stored
 * copies of that dtype with FP32 vectors.  `in` and `out` must not overlap. */
dd_status dd_dirac_apply(dd_gauge* g, dd_dtype dt, int nrhs, const void* in, void* out,
                         void* stream);
/* dd_sap_smooth: x <- SAP(b, x0 = x): p->sap_sweeps sweeps, red then black
 * domains, each domain solved by p->sap_mr_iters even-odd MR iterations
 * (Sec. 2 smoother).  Only sap_sweeps and sap_mr_iters of p are used. */
dd_status dd_sap_smooth(dd_gauge* g, const dd_mg_params* p, dd_dtype dt, int nrhs,
                        const void* b, void* x, void* stream);

/* ---- setup ------------------------------------------------------------------------------
 * dd_setup: random starting vectors from p->seed; dd_setup_from_vectors: the
 * caller's starting vectors (host, canonical complex128 [n][V][4][3]).  Both then
 * run init_sap_apps SAP solves, build (per-aggregate Gram-Schmidt in FP64, P,
 * D_c = P^dag D P, coarse odd-site inverses) and setup_iters adaptive
 * iterations lambda_i <- M lambda_i (Sec. 2).  While D_c is built the setup
 * holds a scratch of FP64 fine vectors, one per column of D_c built in a pass:
 * all 2n columns or 4 GiB of them, or up to half of the budget then free (at
 * most 32 GiB) when that is more.  DD_EBUDGET if even the first figure does
 * not fit; nothing of the setup stays allocated then. */
dd_status dd_setup(dd_gauge* g, const dd_mg_params* p, dd_mg** out);
dd_status dd_setup_from_vectors(dd_gauge* g, const dd_mg_params* p, const double* tv_host,
                                dd_mg** out);
dd_status dd_mg_destroy(dd_mg* mg);
/* Graph mode of the preconditioner M (Eq. 5) inside dd_solve and dd_precond_apply:
 *   0 (default): kernels launched one by one; the host checks the coarse GMRES
 *      between chunks of four Arnoldi steps;
 *   1: the same, each chunk captured once per (nrhs, dtype, position in the
 *      restart cycle) and replayed;
 *   2: all of M (restriction, coarse solve, prolongation, SAP) captured as one
 *      graph per (nrhs, launch and arithmetic choices, input and output buffers)
 *      and replayed, with no host synchronisation: the coarse GMRES decides on
 *      the device which right-hand sides are still active, and the launches of
 *      a step (or cycle) nobody needs return at once.  The graph holds
 *      coarse_max_iters steps, so its cost grows with that cap even when the
 *      solve converges early (an empty launch costs about 2 us).
 * All three give bit-identical results (the masked right-hand sides are never
 * written; mode 2 counts info.coarse_iters_total as the sum over cycles of the
 * longest Arnoldi run).  Graphs hold workspace and buffer addresses and are
 * dropped when the workspace is reallocated.  Kernel timers do not time
 * launches inside graphs (the bytes and flops model of info counts every
 * replay).  Modes 1 and 2 capture on an internal stream on first use; while a
 * capture runs, HIP refuses legacy-stream work and device-wide synchronisation
 * from other threads of the process (dd_gauge_create, dd_setup,
 * dd_mg_release_workspace use them), so threads that overlap such calls with
 * solves should use mode 0.  DD_EINVAL for another mode. */
dd_status dd_mg_set_graphs(dd_mg* mg, int mode);
/* Free the solver workspace of a setup (Krylov bases, scratch vectors and the
 * graphs captured on them); the next solve allocates it again.  For callers
 * that keep many setups resident and solve on one at a time.  Synchronises
 * the device. */
dd_status dd_mg_release_workspace(dd_mg* mg);

/* ---- device footprint --------------------------------------------------------------------
 * The device bytes the library allocates for a problem shape and parameter set,
 * for callers that admit work by HBM budget.  Host arithmetic only: nothing is
 * allocated and no device is touched.
 *   gauge_bytes     : dd_gauge_create plus the storage copies a setup with p adds
 *                     (FP64 links, clover and inverse; FP32 copy; half copy; block tables)
 *   setup_bytes     : what dd_setup keeps resident (P in FP64 and in the storage
 *                     type, working vectors, D_c and odd-site inverses in FP64,
 *                     FP32 and, for half storage, the half type)
 *   scratch_bytes   : the most held on top of those two while dd_gauge_create or
 *                     dd_setup runs, with the Galerkin build at its least column
 *                     chunk (the build takes a larger chunk only out of half of
 *                     the budget then free, so this figure is a sufficient margin)
 *   workspace_bytes : the dd_solve workspace for nrhs right-hand sides
 * DD_ESHAPE / DD_EINVAL as dd_gauge_create and dd_setup would return them. */
typedef struct {
  size_t gauge_bytes, setup_bytes, scratch_bytes, workspace_bytes;
} dd_footprint;
dd_status dd_footprint_bytes(const dd_problem* prob, const dd_mg_params* p, int nrhs, dd_footprint* out);

/* ---- the paper's comparison solver -----------------------------------------------------
 * Sec. 4 "baseline": a mixed-precision nested BiCGstab whose single-precision
 * level is preconditioned by domain decomposition (SAP, N_SAP = 5).  The paper
 * does not give the outer iteration; here it is a defect correction with the
 * FP64 operator (r = b - D x, x += e), and the inner level is an FP32 BiCGstab
 * on D e = r, right preconditioned by SAP over the field's blocks (even-odd
 * minimal-residual domain solves, as in the multigrid smoother), stopped at a
 * relative residual inner_tol.  The paper's domains are 12^4 with SSOR inside;
 * here they are the field's power-of-two blocks.  Right-hand sides advance
 * together; a converged one is not changed any more.  The correction stops with
 * DD_ENOCONV at max_outer_iters or as soon as a step increases the residual of
 * an unconverged right-hand side (x then holds that iterate).  Same vector
 * layout, statuses and info as dd_solve (info.coarse_iters_total = inner steps). */
typedef struct {
  int32_t sap_sweeps;       /* N_SAP (5)                                  */
  int32_t sap_mr_iters;     /* MR steps per domain solve (4)              */
  int32_t inner_max_iters;  /* cap on one inner solve (500)               */
  int32_t max_outer_iters;  /* cap on defect-correction steps (20)        */
  double inner_tol;         /* relative residual of one inner solve (1e-4) */
  dd_dtype store_dtype;     /* operands of the inner level: F32, F16, BF16 */
  int32_t use_x0;           /* 1: x_canon holds the starting guess; 0: start from zero */
} dd_bicgstab_params;
void dd_bicgstab_params_default(dd_bicgstab_params* p);
dd_status dd_solve_bicgstab(dd_gauge* g, const dd_bicgstab_params* p, int nrhs, const double* b_canon_dev,
                            double* x_canon_dev, double tol, dd_solve_info* info, void* stream);

/* ---- autotuner --------------------------------------------------------------------------
 * dd_autotune times every launch-shape candidate of the smoother (waves per
 * SIMD, domain-resident form), the FP64 D apply (workgroup size) and the coarse stencil on matrix
 * cores (sites per workgroup, in the coarse block type the tuning already
 * selects) on this setup's own operators and workspace for nrhs right-hand
 * sides, keeps the fastest in the gauge field (shared by every setup on it)
 * and returns a text report (report may be NULL).  The numerical choices
 * coarse_half, coarse_basis_half and coarse_mfma_half are the caller's and are
 * never changed.  cache_path (may be NULL) names a JSON file of earlier choices
 * keyed by device architecture, lattice, block, n, nrhs, dtypes and coarse
 * block type: a hit applies the stored launch shapes without timing; a miss
 * times and rewrites the file.  Workspace vectors are overwritten; caller data
 * are not touched.
 * dd_gauge_set_tuning / dd_gauge_get_tuning set or read the choice directly
 * (DD_EINVAL for a value outside the lists above). */
dd_status dd_autotune(dd_mg* mg, int nrhs, const char* cache_path, char* report, size_t report_cap);
dd_status dd_gauge_set_tuning(dd_gauge* g, const dd_tuning* t);
dd_status dd_gauge_get_tuning(const dd_gauge* g, dd_tuning* t);
/* "New kappa" (Sec. 4, strange-quark solves): switch the setup to bare mass m0
 * while keeping its test vectors.  Rebuilds the clover term and inverse of the
 * gauge field, then P (same vectors, so the same P), D_c = P^dag D P and the
 * coarse odd-site inverses for the new operator; no adaptive iterations are
 * run.  DD_ESTATE when another dd_mg shares the gauge field; DD_EINVAL for a
 * singular coarse block or non-finite m0. */
dd_status dd_setup_update_mass(dd_mg* mg, double m0);

/* ---- transfer and coarse operator -------------------------------------------------------
 * DD_F64 or DD_F32 vectors.  With DD_F32 the coarse operator is the one the
 * FP32 inner solver uses: FP32 blocks, or, for a setup that stores its operands
 * in a half type and whose gauge field's tuning has coarse_half = 1, FP16 /
 * BF16 blocks rounded from the FP32 copy. */
dd_status dd_restrict(dd_mg* mg, dd_dtype dt, int nrhs, const void* fine_in, void* coarse_out,
                      void* stream);   /* Eq. 3 */
dd_status dd_prolong(dd_mg* mg, dd_dtype dt, int nrhs, const void* coarse_in, void* fine_out,
                     void* stream);    /* Eq. 4 */
dd_status dd_coarse_apply(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out,
                          void* stream);   /* Eq. 2 stencil */
/* approximate D_c^-1: even-odd GMRES to coarse_tol (or coarse_fixed_iters), or, with a third level
 * attached, the level-2 FGMRES cycle (dd_mg_add_level); *iters gets the GMRES (level-2) steps.
 * DD_F64 needs an all-FP64 setup (inner_dtype DD_F64); DD_F32 works on either. */
dd_status dd_coarse_solve(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out,
                          int* iters, void* stream);
/* dd_coarse_solve without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same kernels, same order and the same result as
 * dd_coarse_solve with graphs off.  Its workspace (coarse vectors, Krylov basis,
 * Arnoldi state, reduction partials) is carved from a static per-device scratch
 * array of 128 MiB, held from library load to process exit and not counted
 * against the context's budget; DD_EBUDGET when the call would need more
 * (that is (coarse_restart + 9) coarse vectors of nrhs right-hand sides, plus
 * small state), DD_EINVAL above 64 right-hand sides.  Every call on one GPU
 * shares that array and clears it first: calls that overlap on one GPU (other
 * host threads, other streams) race and must not be issued.  Synchronises
 * `stream` before it returns. */
dd_status dd_coarse_solve_noalloc(dd_mg* mg, dd_dtype dt, int nrhs, const void* in, void* out,
                                  int* iters, void* stream);
/* out = M in (Eq. 5), packed fine vectors of the inner dtype */
dd_status dd_precond_apply(dd_mg* mg, int nrhs, const void* in, void* out, void* stream);

/* ---- third level ---------------------------------------------------------------------------
 * The paper runs two levels and notes that the coarse solver may itself be a
 * multigrid method (Sec. 1, Sec. 2).  dd_mg_add_level applies the construction
 * of Eqs. (1)-(4) once more, to D_c:
 *   - level-2 aggregates are blocks of 2^4 coarse sites; a coarse vector's
 *     chirality s is its components s*n .. s*n + n - 1 (the coarse gamma5 is +1
 *     on the first n components of a site, -1 on the last n);
 *   - P2 holds the n_vec2 level-2 test vectors restricted to each (aggregate,
 *     chirality), orthonormalised there by modified Gram-Schmidt (two sweeps,
 *     vectors in order), so a level-3 site carries 2 n_vec2 components;
 *   - D3 = P2^dag D_c P2 as 9 blocks per level-3 site: block d collects the
 *     coarse hops (x, dd) with x + dd inside the same 2^4 block (d = self) or
 *     crossing its face in direction dd (d = dd), with +mu and -mu kept apart.
 * The coarse correction of M (and dd_coarse_solve) then solves D_c y = b by one
 * cycle of flexible GMRES on D_c (one classical Gram-Schmidt pass per step,
 * at most kcycle_max_iters steps, stopped per right-hand side when its residual
 * estimate reaches kcycle_tol |b|, or exactly kcycle_max_iters steps when
 * kcycle_fixed), right preconditioned by
 *   M2 v = MR_k(D_c; v, x0 = P2 D3^-1 R2 v),
 * k = mr_steps minimal-residual steps on D_c started from the level-3
 * correction, D3^-1 being the even-odd GMRES of the coarse level run on the
 * level-3 lattice (l3_tol / l3_restart / l3_max_iters / l3_fixed_iters; the
 * Gram-Schmidt passes are the setup's coarse_cgs_passes).  Arithmetic is the
 * setup's inner dtype; the level-3 blocks are FP32 (FP64 for an all-FP64 setup).
 * Requires every coarse-lattice extent L[mu] / block[mu] to be a multiple of 4
 * (even level-3 extents, for the even-odd split) and n_vec2 in {6, 8, 12, 16,
 * 20, 24}.  With a third level, graph mode 2 runs as mode 1 (the level-3 GMRES
 * checks convergence on the host), dd_autotune and dd_coarse_solve_noalloc
 * return DD_ESTATE (tune before adding the level), and dd_setup_update_mass
 * rebuilds D3 from the kept P2.  The level's memory is not part of
 * dd_footprint_bytes. */
typedef struct {
  int32_t n_vec2;            /* level-2 test vectors (6, 8, 12, 16, 20 or 24) */
  int32_t setup_iters;       /* test vectors without tv2_host: Gaussian vectors (seed) improved by this many
                                inverse-iteration passes y <- (two-level coarse solve of D_c) y, normalised */
  int32_t mr_steps;          /* minimal-residual steps on D_c after the level-3 correction */
  int32_t kcycle_max_iters;  /* steps of the level-2 FGMRES cycle, 1 .. 64 */
  int32_t kcycle_fixed;      /* 1: exactly kcycle_max_iters steps (no tolerance stop) */
  int32_t l3_restart;        /* level-3 GMRES restart, 1 .. 256 */
  int32_t l3_max_iters;      /* level-3 GMRES iteration cap */
  int32_t l3_fixed_iters;    /* > 0: exactly this many level-3 GMRES steps */
  double kcycle_tol;         /* level-2 relative residual estimate */
  double l3_tol;             /* level-3 relative residual */
  uint64_t seed;             /* Gaussian level-2 test vectors */
} dd_level3_params;
void dd_level3_params_default(dd_level3_params* p);
/* Attach the third level to a setup.  tv2_host: NULL (vectors from the seed and
 * setup_iters) or [n_vec2][Vc][2n] complex128 level-2 test vectors, coarse sites
 * in lexicographic block order (the order of dd_pack_coarse's canonical form),
 * copied.  DD_ESTATE when a level is attached or a stepwise solve holds the
 * workspace, DD_ESHAPE / DD_EINVAL for the limits above, DD_EINVAL when the
 * vectors are rank deficient on some (aggregate, chirality). */
dd_status dd_mg_add_level(dd_mg* mg, const dd_level3_params* p, const double* tv2_host);
dd_status dd_mg_remove_level(dd_mg* mg);   /* back to the two-level coarse solve */
/* Vc3 level-3 sites and 2 n_vec2 components per site (0, 0 without a third level) */
dd_status dd_level3_shape(const dd_mg* mg, int32_t* vc3, int32_t* nc3);
/* Host copies (each pointer may be NULL), level-3 sites X in lexicographic order
 * of the level-3 lattice (x fastest), l = lx + 2 (ly + 2 (lz + 2 lt)) the
 * position of a coarse site inside its block:
 *   tv2 [n_vec2][Vc][2n]        the level-2 test vectors (coarse sites lexicographic)
 *   p2  [Vc3][2][n_vec2][16 n]  P2: entry l*n + c of vector i of chirality s of X
 *   d3  [Vc3][9][nc3][nc3]      D3 blocks, row-major
 * all complex128. */
dd_status dd_export_level3(const dd_mg* mg, double* tv2_host, double* p2_host, double* d3_host);
/* Steps of the last level-2 FGMRES cycle (longest over its right-hand sides) and
 * the level-3 GMRES steps it ran, summed over its preconditioner applications. */
dd_status dd_level3_last(const dd_mg* mg, int32_t* kcycle_steps, int32_t* l3_steps);

/* ---- solve -------------------------------------------------------------------------------
 * FGMRES(m) right-preconditioned by M; the outer residual, orthogonalisation
 * and Hessenberg least squares are FP64 on the device; stops when every
 * right-hand side has |b - D x| / |b| <= tol with the FP64 operator.
 * b and x: canonical complex128 device buffers [nrhs][V][4][3]; info: nrhs entries. */
dd_status dd_solve(dd_mg* mg, int nrhs, const double* b_canon_dev, double* x_canon_dev,
                   double tol, dd_solve_info* info, void* stream);

/* ---- stepwise solve ----------------------------------------------------------------------
 * The same FGMRES(m) as dd_solve (which is begin, add every right-hand side,
 * step until no slot runs, take every slot, end), driven one restart cycle at a
 * time, for a server that admits right-hand sides into a running batch at the
 * restart boundaries and hands results back as they finish.
 *
 * A state holds `capacity` slots, each free, running or done.  Every launch of
 * a step covers slots [0, highest running slot]; reductions, masks and
 * Hessenberg data are per slot, so a right-hand side gets bit-identical results
 * whether it runs alone or beside others and whenever it joins.  The iteration
 * cap max_outer_iters is applied per slot at restart boundaries (a cycle is
 * shortened so the longest-running slot stops at the cap).
 *
 * dd_solve_begin: allocate (or reuse) the workspace for `capacity` right-hand
 *   sides; tol as in dd_solve.  One live state per dd_mg (they share its
 *   workspace).  DD_EBUDGET/DD_ENOMEM as dd_solve.
 * dd_solve_add: start slot `slot` (must be free) from x = 0 on the canonical
 *   complex128 device vector b [V][4][3] (read before the call returns).
 *   A zero b is done at once (x = 0, converged); non-finite b gives DD_ENAN
 *   and leaves the slot free.  Synchronises the state's stream.
 * dd_solve_step: one restart cycle of the running slots, then their
 *   true-residual check: a slot whose |b - D x| / |b| <= tol (FP64 operator),
 *   or that reached max_outer_iters, becomes done.  slot_state (capacity
 *   int32 entries, may be NULL) receives 0 free, 1 running, 2 done.  DD_ENAN
 *   on breakdown.  A step with no running slot does nothing.  Synchronises
 *   the state's stream.
 * dd_solve_take: copy a done slot's solution to the canonical complex128
 *   device buffer x [V][4][3], fill info (may be NULL; t_solve_s counts from
 *   dd_solve_begin, coarse_iters_total and the work model cover every slot of
 *   the state so far) and free the slot.  DD_ESTATE if the slot is not done.
 * dd_solve_end: release the state (not the workspace, which the dd_mg keeps). */
typedef struct dd_solve_state dd_solve_state;
dd_status dd_solve_begin(dd_mg* mg, int capacity, double tol, void* stream, dd_solve_state** out);
dd_status dd_solve_add(dd_solve_state* s, int slot, const double* b_canon_dev);
dd_status dd_solve_step(dd_solve_state* s, int32_t* slot_state);
dd_status dd_solve_take(dd_solve_state* s, int slot, double* x_canon_dev, dd_solve_info* info);
dd_status dd_solve_end(dd_solve_state* s);

/* ---- exports for parity checks (host buffers) ----------------------------------------- */
dd_status dd_export_maps(const dd_gauge* g, int32_t* agg_of_site, int32_t* local_of_site,
                         int32_t* packed_index_of_site, int8_t* color_of_block);
dd_status dd_export_clover(const dd_gauge* g, double* clover_host /* [V][2][36] */,
                           double* clover_inv_host /* [V][2][36] */);
/* raw stored operand copies of dtype dt, in the packed layout: links [4][9][V]
 * pairs and clover [36][V] pairs of that dtype (16, 8, 4 or 4 bytes per pair);
 * sites in packed order (dd_export_maps gives packed_index_of_site) */
dd_status dd_export_operands(dd_gauge* g, dd_dtype dt, void* links_host, void* clover_host);
dd_status dd_export_coarse(const dd_mg* mg, double* dc_host /* [Vc][9][2n][2n] c128 */);
dd_status dd_export_vectors(const dd_mg* mg, double* tv_host /* [n][V][4][3] c128 */);

/* ---- per-kernel timing (benchmark support) -----------------------------------
 * Brackets every launch of the named kernel ("*" = all instrumented kernels:
 * k_dirac, k_sap_colour, k_restrict, k_prolong, k_coarse_mv, k_dots,
 * k_multi_axpy) with HIP events on its launch stream and records the launch's
 * algorithmic bytes and flops.  NULL disables timing and clears the records. */
dd_status dd_kernel_timer_enable(const char* name);
dd_status dd_kernel_timer_read(const char* name, double* total_ms, int64_t* launches, double* bytes,
                               double* flops);
dd_status dd_kernel_timer_names(char* buf, size_t cap);

#ifdef __cplusplus
}
#endif
#endif
