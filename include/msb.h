/*
 * msb.h -- C ABI of the MI355X multi-shifted BiCG library for resonant
 * (Kramers-Heisenberg) spectra.
 *
 * Problem (paper Eqs. kramers1 and intermediateState, shifted form of
 * Appendix A, Eq. shifted_linear_eq):
 *
 *   (A - w_in I) Psi(w_in) = E,   A = H' - E_G - i Gamma,   E = O2 |G>,
 *   I(w_in, w) = (1/pi) Im <phi| (H - E_G - w - i eta)^{-1} |phi>,  phi = O1 Psi.
 *
 * H is the single-band Hubbard model (Sec. III, Eq. Hubbard) on an arbitrary
 * bond list; H' adds the core-hole potential U_c on one site (valence part of
 * Eq. intermediate_H).  All shifts of one right-hand side are solved from a
 * single Krylov space by the multi-shift complex-symmetric BiCG of
 * Appendix D (Algorithm 1) with one matrix-vector product per iteration
 * (Appendix A's r~ = r* simplification).
 *
 * Conventions shared by every call
 * --------------------------------
 * Basis / layout.  Fixed (N_up, N_dn) sector, D = C(L,N_up) * C(L,N_dn).
 *   Index = rank_up(u) * n_dn + rank_dn(d), where u, d are L-bit occupation
 *   strings and rank is the position among L-bit integers with the same
 *   popcount in ascending order.  Kets are c+_{o1} c+_{o2} ... |0> with all
 *   spin-up orbitals (site order) before all spin-down orbitals.
 * Vectors.  Device pointers; complex numbers interleaved (re, im):
 *   MSB_C128 = two doubles, MSB_C64 = two floats.  Multi-vector arguments
 *   are row-major with the element index fastest, e.g. psi[sys][shift][D].
 * Ownership.  The caller allocates and owns every vector argument; the
 *   library never frees or retains them.  The library owns the context:
 *   basis tables, workspace and captured graphs, released by msb_destroy.
 *   Inputs are never modified.
 * Streams.  `stream` is a hipStream_t of the HIP runtime this library is
 *   linked against (one made by msb_stream_create, or any other stream of
 *   that runtime), or NULL for that runtime's null stream.  Every call first
 *   orders itself after the work already queued on `stream`: calls that run
 *   on `stream` itself (msb_apply, msb_apply_timed, msb_number_op,
 *   msb_dipole, msb_combine, msb_spectrum, msb_ground_state, msb_autotune)
 *   enqueue behind it, and calls that run on the context's own streams
 *   (msb_solve, msb_solve_reseed, msb_mlp_train, msb_mlp_predict) wait for it with
 *   hipStreamSynchronize before they start.  Calls are blocking: they return
 *   after all of their device work has completed, so outputs are ready on
 *   any stream.  A stream of another HIP runtime instance (a framework that
 *   bundles its own runtime, such as a ROCm build of PyTorch) is not a valid
 *   handle here: synchronise it and pass NULL.
 * Errors.  Every call returns an msb_status; msb_last_error() returns a
 *   thread-local message for the last failure on the calling thread.
 * Threads.  A context may be used by one thread at a time.
 */
#ifndef MSB_H
#define MSB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MSB_MAX_BOND_TYPES 8

typedef struct msb_ctx msb_ctx;

typedef enum {
  MSB_OK = 0,
  MSB_EINVAL = 1,         /* invalid argument (message says which) */
  MSB_ENOMEM = 2,         /* device memory footprint exceeds what is free */
  MSB_EHIP = 3,           /* a HIP runtime call failed */
  MSB_BREAKDOWN = 4,      /* |r^T A p| fell below 1e-14 |r||Ap| (COCG breakdown) */
  MSB_NOT_CONVERGED = 5,  /* iteration cap reached before every shift converged */
  MSB_FLOOR = 6           /* MSB_C64: a residual replacement found the recurrence residual more than
                             10x below the true one, i.e. the complex64 recurrence reached its
                             attainable accuracy before every shift met tol; that system stops there */
} msb_status;

typedef enum { MSB_C128 = 0, MSB_C64 = 1 } msb_prec;

/* Lattice model H (Eq. Hubbard):
 *   H = -sum_b t_b sum_sigma (c+_{j_b sigma} c_{i_b sigma} + h.c.) + U sum_i n_{i up} n_{i dn}.
 * Host arrays of length n_bonds; each unordered pair should appear once.
 * Bonds with equal t form one "bond type" (types numbered by first
 * appearance, at most MSB_MAX_BOND_TYPES); per-system amplitudes may
 * override a type's t (msb_system.t_amp).
 * Directed bonds (bond_t_rev != NULL): the hop term of bond b is
 *   -sum_sigma (t_b c+_{j_b sigma} c_{i_b sigma} + t_rev_b c+_{i_b sigma} c_{j_b sigma}),
 * non-symmetric where t_rev_b != t_b (non-reciprocal, dissipative models).
 * Every distinct pair (t, t_rev) is a class k with two types, 2k for the hop
 * i -> j (amplitude t) and 2k + 1 for j -> i (t_rev), so at most
 * MSB_MAX_BOND_TYPES / 2 classes; per-system t_amp may make any system
 * non-symmetric, and msb_solve then uses the dual-space form.
 * Limits: 2 <= n_sites <= 20, C(L, N_sigma) <= 65535. */
typedef struct {
  int n_sites, n_up, n_dn, n_bonds;
  const int* bond_i;
  const int* bond_j;
  const double* bond_t;
  double U;
  const double* bond_t_rev;   /* NULL: t_rev = t (symmetric hopping) */
} msb_model;

/* One linear system / Hamiltonian instance on the context's sector.
 *   H'_s = H(U_s, t_amp_s) + Uc_s (n_{j up} + n_{j dn}),  j = core_site_s,
 *   A_s  = H'_s - E_G_s - i Gamma_s.
 * core_site = -1 means no core hole (H' = H).  U = NaN keeps the model's U.
 * n_amp = 0 keeps the model's bond amplitudes; otherwise t_amp[0..n_amp-1]
 * replace the amplitudes of bond types 0..n_amp-1. */
typedef struct {
  int core_site;
  double Uc;
  double E_G;
  double Gamma;
  double U;
  int n_amp;
  double t_amp[MSB_MAX_BOND_TYPES];
} msb_system;

/* Per-solve report (msb_solve).  Pointer members are optional host arrays
 * (NULL = not wanted) of length nsys*n_shift (index sys*n_shift + shift) or nsys. */
typedef struct {
  int iters;             /* seed iterations of the longest system (= its matrix-vector products) */
  int mvms;              /* seed matrix-vector products summed over systems */
  int breakdown_iter;    /* first iteration with breakdown, -1 if none */
  int flushes;           /* multi-shift assembly passes performed */
  int* sys_iters;        /* [nsys] iterations of each system */
  int* shift_iters;      /* [nsys*n_shift] iteration at which the shift froze, -1 = not converged */
  double* resid_rec;     /* [nsys*n_shift] recurrence residual |r_m| / |zeta_m| / |E| */
  double* resid_true;    /* [nsys*n_shift] FP64 true residual |E - (A - w)Psi| / |E| (extra applies) */
  double t_iter_ms;      /* device time of the seed iterations */
  double t_flush_ms;     /* device time of the multi-shift assembly */
  double t_true_ms;      /* device time of the true-residual check */
  double t_gemm_ms;      /* device time of the dense assembly launches alone */
  int n_gemm;            /* number of dense assembly launches */
  double gemm_flops;     /* algorithmic flops of those launches: 8 D sum(range lengths) */
  double gemm_bytes;     /* algorithmic bytes: residual slots read + outputs written (+read) */
  int replacements;      /* residual replacements performed, summed over systems (MSB_C64 only) */
  double* seed_hist;     /* optional [nsys*hist_len]: |r_m| / |E| of the seed for m < hist_len
                            (the replaced value at a replacement), NaN after the last iteration */
  int hist_len;
  int apply_threads;     /* launch shape of the seed apply: threads per workgroup, */
  int apply_ept;         /*   elements of a row per thread, */
  int apply_nv;          /*   systems per workgroup, */
  int apply_passes;      /*   1, or 2 / 3 when the up-spin hops ran as a separate column-panel
                            pass (3: panels staged in LDS), */
  int apply_order;       /*   row order: 0 contiguous rank range per XCD, 1 level order */
  double t_setup_ms;     /* host wall time before the workspace: validation, apply tuning, planning */
  double t_alloc_ms;     /* host wall time of (re)allocating the workspace (0 when reused) */
  double t_wall_ms;      /* host wall time of the whole call */
  int apply_panel_width; /* columns of the seed apply's LDS panel (passes 3), else 0 */
  int group;             /* systems iterated together: the batch ran in groups of this many */
  int bank_slots;        /* residual slots per system in the bank (a flush when they are full) */
} msb_info;

/* One launch shape of the Hamiltonian apply and its measured time. */
typedef struct {
  int threads;           /* threads per workgroup (one workgroup per up-spin row) */
  int elems_per_thread;  /* threads * elems_per_thread >= number of down-spin states */
  int vectors;           /* systems handled by one workgroup (they share the hop tables) */
  int passes;            /* 1: one row kernel; 2: diagonal and up-spin hops first, on column
                            panels that stay in one XCD's L2, then the row kernel adds the
                            down-spin hops in place; 3: the same with each column panel
                            (every up-spin row, panel_width columns) staged in LDS (neither
                            is used by the residual check) */
  int row_order;         /* 0: each XCD walks one contiguous range of up-spin ranks of every
                            system; 1: the rows of all systems in level order (ascending sum
                            of occupied site indices), one contiguous eighth per XCD */
  int panel_width;       /* passes = 3: down-spin columns of one LDS-staged panel (else 0) */
  double ms;             /* mean time of one apply of min(nsys, 16) vectors (msb_autotune) */
} msb_shape;

/* Tuning knobs of msb_solve; pass NULL for defaults. */
typedef struct {
  int chunk;             /* seed iterations per captured graph launch (default 16) */
  int bank_slots;        /* residual slots kept before a flush; 0 = min(maxit + 1, 1024) */
  int batch;             /* systems iterated together (block apply), at most; 0 = no limit.  The
                            whole batch runs together when every system's bank holds
                            `bank_slots` slots; otherwise it runs in the largest groups whose
                            banks hold min(bank_slots, 512) slots each (a flush before the
                            last iteration also assembles the search directions), and only
                            when no group does, all together with the largest bank that fits */
  int replace_every;     /* MSB_C64 only: the seed residual is replaced by E - A_s x_m (x_m and the
                            product in complex128) at the first chunk boundary at least
                            `replace_every` iterations after the previous replacement (a bank
                            restart moves the boundaries), while |r_m| > max(tol, 1e-12) |E|;
                            0 = default 50, < 0 = off.  When it is on and `chunk` is 0, the
                            chunk is min(replace_every, 64). */
  int use_graph;         /* 0 or 1 = capture the chunk in a hipGraph (default), -1 = plain launches */
  double mem_fraction;   /* fraction of free device memory the workspace may use (default 0.9) */
  int assembly_engine;   /* multi-shift assembly: 0 = the default: the FP64 vector ALU with
                            three real products per complex product, except for an MSB_C64
                            bank with 128 or more shifts, which takes 5; 1 = FP64 matrix
                            cores, four products; 2 = FP64 vector ALU, four products; 3 = as
                            0 with 64 shifts per workgroup; 4 = as 0 with 256 elements and
                            eight wavefronts of four shifts; 5 = int8 matrix cores on 8-bit
                            digit planes of the operands (six planes, 46 bits, for an
                            MSB_C128 bank; five planes, 38 bits, for MSB_C64); 6 = FP64
                            matrix cores with three products, the bank staged in LDS
                            (MSB_C128 only: MSB_C64 takes the vector ALU); 7 = the FP64
                            vector ALU with three products in every case */
  int autotune;          /* 0 = tune the apply shape on first use (default), -1 = default shape
                            unless one was tuned or pinned before */
  int dual;              /* 0 = the dual-space (BiCG) form only when some system's A is not
                            symmetric (default), 1 = always; MSB_C128 only */
  int direct_ap;         /* 0 = (default) in MSB_C128 (not in the dual form) the seed applies A
                            to its residual r_m in place and forms
                            A p_m = A r_m + beta_{m-1} A p_{m-1} in the same pass; MSB_C64 forms
                            p_m and applies A to it (Algorithm 1 as written); 1 = that direct
                            form in both precisions.  Other values: MSB_EINVAL (a product
                            carried in complex64 storage drifts from A p_m) */
  int interleave;        /* 1 = in the direct seed form, batches of two or more systems keep p and
                            A p with the systems of a group of 4 (or 2) interleaved element by
                            element and run the two-pass block apply of msb_apply_block (one
                            neighbour-row gather per group); 0 or -1 = (default) one vector per
                            system (measured faster on the workloads here) */
} msb_opts;

/* ---- context -------------------------------------------------------------- */

/* Builds the basis and the per-spin hopping tables (Jordan-Wigner signs of
 * Eq. Hubbard) on the host and uploads them to the current device.
 * Limits: 2 <= n_sites <= 20; one down-spin row (C(n_sites, n_dn) states) is
 * staged in one workgroup's LDS, so 8 * C(n_sites, n_dn) bytes must fit it
 * (160 KB on gfx950: up to 20480 states; complex128 applies need 16 bytes per
 * state, up to 10240 states, and return MSB_EINVAL beyond).
 * Errors: MSB_EINVAL for sizes outside the limits; MSB_EHIP on upload failure. */
msb_status msb_create(const msb_model* model, msb_ctx** out);
void msb_destroy(msb_ctx* ctx);
/* Frees the context's solve / spectrum workspace (the next call that needs it
 * allocates it again), e.g. before a caller allocates large buffers of its
 * own.  Waits for the context's stream first.  Errors: MSB_EINVAL for a null
 * context; MSB_EHIP if the wait or the free fails. */
msb_status msb_release_workspace(msb_ctx* ctx);
int64_t msb_dim(const msb_ctx* ctx);
/* Per-spin sector sizes and bond-type count (any pointer may be NULL). */
msb_status msb_sector_info(const msb_ctx* ctx, int* n_up_states, int* n_dn_states, int* n_bond_types);
const char* msb_last_error(void);
/* 1 if the library was built for and found a gfx950 device. */
int msb_device_ok(void);
/* A default-priority, non-blocking stream of the library's HIP runtime on the
 * current device, for callers that have no stream of that runtime; release
 * it with msb_stream_destroy (after the last call that uses it).
 * Errors: MSB_EINVAL for a null `out`; MSB_EHIP if the runtime refuses. */
msb_status msb_stream_create(void** out);
msb_status msb_stream_destroy(void* stream);

/* ---- operators -------------------------------------------------------------- */

/* y_s = (H'_s - E_G_s - i Gamma_s - shift) x_s for s < nsys (matrix-free
 * Kronecker apply: H_up (x) I + I (x) H_dn + diagonal).  x, y: [nsys][D] of
 * `prec`; x and y must not overlap. */
msb_status msb_apply(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                     msb_prec prec, const void* x, void* y, void* stream);

/* Timing helper for the apply above: `reps` back-to-back launches on `stream`
 * bracketed by HIP events; *ms_per_apply receives the mean launch duration.
 * Same arguments and errors as msb_apply; reps >= 1. */
msb_status msb_apply_timed(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                           msb_prec prec, const void* x, void* y, int reps,
                           double* ms_per_apply, void* stream);

/* The block apply (SpMM) of the batched form: y_s = (H'_s - E_G_s - i Gamma_s - shift) x_s
 * for s < nsys, with the vectors of each group of `group` (2 or 4) systems
 * interleaved element by element: x, y are [ceil(nsys / group)][D][group]
 * (element i of system s at (s / group * D + i) * group + s % group), so one
 * gather of a neighbour row serves the whole group.  Runs as two passes
 * (column panels for the diagonal and H_up (x) I, rows staged in LDS for
 * I (x) H_dn); y is written in full for the nsys systems (the slots of a
 * ragged last group are not).  With ms_per_apply != NULL, `reps` more applies
 * are timed with HIP events and their mean is returned.
 * Errors: MSB_EINVAL for group not 2 or 4, nsys < group, or rows of `group`
 * systems that do not fit a workgroup's LDS (MSB_C64: D's row of up to 5119
 * states for groups of 4; MSB_C128: 2559), and as msb_apply. */
msb_status msb_apply_block(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                           msb_prec prec, int group, const void* x, void* y, int reps,
                           double* ms_per_apply, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the apply
 * of msb_apply with no allocation at all.  The per-system parameters are
 * staged in a fixed device array of the library (MSB_NOALLOC_MAX_SYS systems,
 * about 104 bytes each; one copy per GPU, set up by msb_create and held until
 * the process ends); the launch shape is the one tuned or pinned before for
 * this (system count, precision), else the default shape -- no tuning runs.
 * Same arguments and results as msb_apply.  Every call on one GPU shares that
 * GPU's staging array, so calls that overlap on one GPU (other threads, other
 * contexts) race: serialise them.
 * Errors: MSB_EINVAL for nsys outside [1, MSB_NOALLOC_MAX_SYS] and as msb_apply;
 * MSB_EHIP if the staging array of the context's device was not set up. */
#define MSB_NOALLOC_MAX_SYS 1024
msb_status msb_apply_noalloc(msb_ctx* ctx, const msb_system* sys, int nsys, double shift,
                             msb_prec prec, const void* x, void* y, void* stream);

/* y = (w_up n_{site up} + w_dn n_{site dn}) x, or y = x if site < 0 (the
 * sector-preserving operators O1 / O2 used by the workloads).
 * x: [count][D] real FP64 (x_real != 0) or C128; y: [count][D] C128. */
msb_status msb_number_op(msb_ctx* ctx, int site, double w_up, double w_dn, int count,
                         int x_real, const void* x, void* y, void* stream);

/* ---- ground state (precondition of Eq. intermediateState) ----------------- */

/* Lowest eigenpair of H(sys->U, sys->t_amp) by FP64 Lanczos with full
 * reorthogonalisation from the caller's start vector x0 (real, [D]); the
 * tridiagonal problem is solved on the host by bisection + inverse iteration.
 * Stops when the Ritz residual |b_k y_k| <= tol |E_G| or at maxit.
 * G: [D] real FP64 output, unit norm, sign fixed so that sum(G) >= 0.
 * Errors: MSB_NOT_CONVERGED at maxit (E_G, G hold the last Ritz pair). */
msb_status msb_ground_state(msb_ctx* ctx, const msb_system* sys, const double* x0,
                            double tol, int maxit, double* E_G, double* G,
                            int* iters, void* stream);

/* Dipole-type operators that add or remove one valence electron (Sec. III:
 * O_2 creates the electron the x-ray promotes, O_1 removes one on emission):
 *   y[v] = sum_j coef_j c+_{j spin} x[v]   (create = 1)
 *   y[v] = sum_j coef_j c_{j spin} x[v]    (create = 0),   v < nvec.
 * x lives in the sector of `src`; y in the sector of `dst`, which must be the
 * same lattice with (N_up +- 1, N_dn) for spin 0 or (N_up, N_dn +- 1) for
 * spin 1.  Jordan-Wigner order: all up orbitals (sites 0..L-1) before all
 * down orbitals, so c+_{j s} on a basis state carries (-1)^{number of occupied
 * orbitals before (j, s)} -- the order the Hamiltonian's hop signs assume.
 * coef: host [2 * n_sites] complex (re, im); x: [nvec][D_src] C128, y:
 * [nvec][D_dst] C128 (device; overwritten, or added to when accumulate != 0,
 * which forms coherent site sums such as sum_j e^{iqj} c_{j s} Psi_j one site
 * at a time).  Errors: MSB_EINVAL for mismatched lattices or sectors, spin
 * not 0/1, nvec outside 1..65535. */
msb_status msb_dipole(const msb_ctx* src, const msb_ctx* dst, int spin, int create,
                      const double* coef, int nvec, int accumulate, const void* x, void* y,
                      void* stream);

/* ---- the hot path: all shifts of every system from one Krylov space ------- */

/* Multi-shift COCG (Algorithm 1, corrected reading: (1 - alpha_m w) in the
 * zeta recurrence, beta_{m-1} in the shift formulas, bilinear r^T r products).
 * For each system s and shift k:
 *   (A_s - w_in[k] I) psi[s][k] = E[s].
 * E: [nsys][D] C128 (any complex vector; E^T E != 0).  psi: [nsys][n_shift][D] of `prec`.
 * The seed system is A_s - seed_shift I.  Shift k freezes once
 * |r_m| / |zeta_m(w_k)| <= tol |E_s|.  MSB_C64 runs the vectors in complex64
 * with FP64 reductions and scalars, and replaces the seed residual by the
 * FP64 true residual every opts->replace_every iterations (the seed solution
 * x_m that needs is rebuilt in FP64 from the residual bank at each replacement).
 * In MSB_C128 the seed by default carries A p_m by recurrence
 * (opts->direct_ap): the apply reads r_m in place from the residual bank and
 * writes A p_m = A r_m + beta_{m-1} A p_{m-1} over the previous product, so
 * no separate update of p_m runs; sigma_m = r_m^T A p_m and every scalar are
 * as in Algorithm 1, the iterates equal up to rounding.
 * When some system's A is not symmetric (directed bonds with different
 * amplitudes, msb_model) the dual-space form runs instead: a shadow residual
 * r~ and direction p~ follow the same recurrences with A^T (a second apply per
 * iteration), sigma = r~^T A p and rho = r~^T r; the shift recurrences are
 * unchanged.  It needs MSB_C128 (MSB_EINVAL otherwise); opts->dual = 1 forces
 * it for symmetric systems too (then r~ = r and the iterates are identical).
 * msb_ground_state and msb_spectrum need symmetric systems.
 * The seed also stops when its residual falls below 1e-150 |E_s| with shifts
 * still open (its bilinear products would leave the float64 range; a seed far
 * from the resonances converges much faster than the shifts it carries).
 * Returns MSB_NOT_CONVERGED (psi holds the last iterates; cap reached or seed
 * exhausted), MSB_FLOOR (MSB_C64
 * only; psi holds the iterates at the attainable accuracy, shifts that had not
 * met tol have shift_iters = -1 and their resid_true says what was reached) or
 * MSB_BREAKDOWN (psi holds the iterates before the breakdown).  Precedence when
 * systems end differently: BREAKDOWN, NOT_CONVERGED, FLOOR.
 * Footprint (checked before launching): about (bank_slots + 6) * D * s * batch
 * (+ 2 n_shift D s batch when the bank must be flushed mid-solve). */
msb_status msb_solve(msb_ctx* ctx, const msb_system* sys, int nsys, const void* E,
                     const double* w_in, int n_shift, double seed_shift, double tol,
                     int maxit, msb_prec prec, void* psi, msb_info* info,
                     const msb_opts* opts, void* stream);

/* Adaptive reseeding (Appendix E) around msb_solve, one system at a time.
 * Round 0 solves every shift of system s from seed_shift.  After each round,
 * a shift of that round fails when its FP64 true residual |r_t(w)| / |E_s|
 * exceeds reseed_tol or it never froze.  (For a frozen shift the paper's
 * collinearity deviation |r_t(w) - r_m / zeta_m(w)| differs from |r_t(w)| by
 * at most tol |E_s|, so reseed_tol should be well above tol.)  The failing
 * shift with the largest true residual becomes the seed and only the failing
 * shifts are solved again from r_0 = E_s; at most max_rounds rounds in all.
 * E: [nsys][D] C128; psi: [nsys][n_shift][D] of prec (device).  Host outputs
 * (each may be NULL): seed_of [nsys][n_shift] the seed whose solve gave each
 * final psi row, resid_true [nsys][n_shift] the final true residuals,
 * rounds [nsys] the rounds used.  opts applies to every inner solve.
 * Returns MSB_OK when every shift passes, MSB_NOT_CONVERGED when some still
 * fail after max_rounds, MSB_EINVAL for bad arguments (reseed_tol <= 0,
 * max_rounds < 1), or the first MSB_ENOMEM / MSB_EHIP of an inner solve. */
msb_status msb_solve_reseed(msb_ctx* ctx, const msb_system* sys, int nsys, const void* E,
                            const double* w_in, int n_shift, double seed_shift, double tol,
                            int maxit, msb_prec prec, double reseed_tol, int max_rounds,
                            void* psi, double* seed_of, double* resid_true, int* rounds,
                            const msb_opts* opts, void* stream);

/* Autotuner of the Hamiltonian apply (the block SpMM of the batched form).
 * Times every compiled launch shape usable for this context's row length with
 * min(nsys, 16) systems in `prec` on scratch vectors (HIP events: one warm-up
 * and one timed apply each, four more for shapes within 1.5x of the best so
 * far; the reported time is the mean of the timed ones), keeps the fastest in the context for every later apply of that
 * (nsys class, prec), and reports the table (out may be NULL).  msb_solve,
 * msb_apply, msb_apply_timed, msb_ground_state and msb_spectrum tune on their
 * first use of a (nsys class, precision) unless opts->autotune = -1.
 * Errors: MSB_ENOMEM if the scratch vectors do not fit. */
msb_status msb_autotune(msb_ctx* ctx, int nsys, msb_prec prec, msb_shape* out, int max_out,
                        int* n_out, void* stream);
/* Pins the apply shape for (min(nsys, 16), prec); shape->threads == 0 returns
 * to the default shape.  Errors: MSB_EINVAL if the shape is not usable here. */
msb_status msb_set_shape(msb_ctx* ctx, int nsys, msb_prec prec, const msb_shape* shape);

/* phi[k] = sum_s phase_s * O1_s psi[s][k]  for k < n_shift, with
 * O1_s = (w_up n_{site up} + w_dn n_{site dn}) or identity when o1_site[s] < 0.
 * psi: [nsys][n_shift][D] of `prec`; phi: [n_shift][D] C128.
 * phase_re/phase_im/o1_site/o1_wup/o1_wdn: host arrays [nsys] (o1_* may be NULL = identity). */
msb_status msb_combine(msb_ctx* ctx, int nsys, int n_shift, msb_prec prec, const void* psi,
                       const double* phase_re, const double* phase_im, const int* o1_site,
                       const double* o1_wup, const double* o1_wdn, void* phi, void* stream);

/* Kramers-Heisenberg intensity by a Lanczos continued fraction per vector
 * (Eq. kramers1 with 0+ -> eta):
 *   I[k][j] = (1/pi) Im <phi_k| (H - E_G - w[j] - i eta)^{-1} |phi_k>.
 * H = H(sys->U, sys->t_amp) (core_site, Uc, Gamma ignored); E_G = sys->E_G.
 * All n Lanczos recurrences run together as a block; each stops when
 * max_j |I_k - I_{k-10}| / max_j I_k < cf_tol, its Lanczos vector vanishes,
 * or lanczos_max steps.  phi: [n][D] C128; w: host [n_w]; I: host [n][n_w];
 * depth: host [n] (may be NULL). */
msb_status msb_spectrum(msb_ctx* ctx, const msb_system* sys, const void* phi, int n,
                        const double* w, int n_w, double eta, int lanczos_max,
                        double cf_tol, double* I, int* depth, void* stream);

/* msb_spectrum that also returns the continued fraction it evaluated
 * (Lanczos tridiagonalisation of H from each phi_k):
 *   G_k(z) = b_0^2 / (z - a_0 - b_1^2 / (z - a_1 - b_2^2 / ...)),
 *   a_i = <q_i|H|q_i>,  b_0 = |phi_k|,  b_i = |H q_{i-1} - a_{i-1} q_{i-1} - b_{i-1} q_{i-2}|
 * with q_0 = phi_k / |phi_k| (a_0 and b_0^2, b_1^2 are the first spectral
 * moments).  a, b: host [n][ld]; entries i < min(depth[k], ld) are written,
 * the rest set to 0.  depth: host [n] (required).  Other arguments and errors
 * as msb_spectrum; MSB_EINVAL if a, b or depth is NULL or ld < 1. */
msb_status msb_spectrum_cf(msb_ctx* ctx, const msb_system* sys, const void* phi, int n,
                           const double* w, int n_w, double eta, int lanczos_max,
                           double cf_tol, double* I, int* depth, double* a, double* b, int ld,
                           void* stream);

/* ---- learned form: ensemble surrogate I(U, t', U_c, Gamma, w_in, w) --------
 * Not part of the paper's method: a regression network beside the solver,
 * trained on spectra the solver produced, with the solver as fallback.
 * Each member is a perceptron 6 -> 512 -> 512 -> 512 -> 1 with GELU
 * (x Phi(x), exact normal CDF) between the layers.  Inputs are normalised
 * as (x - in_shift) * in_scale feature by feature; the network output is
 * out_scale * I.  The two 512 x 512 layers run on bfloat16 matrix cores with
 * float32 accumulation; their operands (weights, activations, back-propagated
 * gradients) are rounded to bfloat16, all other arithmetic and the master
 * weights are float32.  Parameters of one member are a flat float32 vector of
 * msb_mlp_num_params() values: W1[6][512] b1[512] W2[512][512] b2[512]
 * W3[512][512] b3[512] W4[512] b4 (weights [in][out]).  Device arrays are
 * caller-owned; every call is blocking. */
typedef struct msb_mlp msb_mlp;
int64_t msb_mlp_num_params(void);
/* members in [1, 64]; parameters start at zero (set them before use).
 * Errors: MSB_EINVAL for bad arguments, MSB_EHIP on allocation failure. */
msb_status msb_mlp_create(int members, const double in_shift[6], const double in_scale[6],
                          double out_scale, msb_mlp** out);
void msb_mlp_destroy(msb_mlp* mlp);
/* Host float32 [msb_mlp_num_params()] in/out; set also clears Adam's moments
 * and step count. */
msb_status msb_mlp_set_params(msb_mlp* mlp, int member, const float* params);
msb_status msb_mlp_get_params(const msb_mlp* mlp, int member, float* params);
/* Loss mean((out - out_scale T)^2) over n points and its gradient (host float32
 * [msb_mlp_num_params()]) for one member.  X: device float32 [n][6]; T: device
 * float32 [n]; 1 <= n <= 131072. */
msb_status msb_mlp_grad(msb_mlp* mlp, int member, const float* X, const float* T, int n,
                        double* loss, float* grad);
/* `steps` Adam steps (lr; beta 0.9, 0.999; eps 1e-8) of every member at once.
 * Step s of member m uses the points perm[m][s * batch ... (s + 1) * batch)
 * (device int32 [members][steps * batch], indices < n_points).  batch: a
 * multiple of 128 up to 131072.  loss_hist (optional host [members][steps])
 * receives each step's loss.  One step is captured in a hipGraph and replayed. */
msb_status msb_mlp_train(msb_mlp* mlp, const float* X, const float* T, int64_t n_points,
                         const int* perm, int batch, int steps, double lr, double* loss_hist,
                         void* stream);
/* Ensemble mean and standard deviation (over members, population) of I at n
 * points.  X: device float32 [n][6]; mean, sd: device float32 [n]. */
msb_status msb_mlp_predict(msb_mlp* mlp, const float* X, int64_t n, float* mean, float* sd,
                           void* stream);
/* Solver fallback rule (host arrays): row r of an [n_rows][n_cols] (w_in, w)
 * grid falls back when sd exceeds frac * max(mean) anywhere in the row. */
msb_status msb_mlp_fallback(const float* mean, const float* sd, int n_rows, int n_cols, double frac,
                            int* row_mask);

#ifdef __cplusplus
}
#endif
#endif /* MSB_H */
