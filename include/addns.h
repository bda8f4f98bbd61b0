/*
 * libaddns -- algebraic non-overlapping domain decomposition preconditioner
 * inside restarted (F)GMRES for block 2x2 saddle-point (Oseen) systems,
 * native to AMD Instinct MI355X (gfx950).
 *
 * The method (Kumar, "Purely algebraic domain decomposition methods for the
 * incompressible Navier-Stokes equations"):
 *   - the matrix is the only input (section 1: the method takes the matrix
 *     and right-hand side as its input); rows are scaled by their largest
 *     absolute entry (section 5);
 *   - a graph partition gives P^T C P = [D E; F G], D = blkDiag(A_11..A_mm)
 *     (section 1; section 3.3);
 *   - mini Schur complements S_i = G_i - F_i D_{r_i}^{-1} E_i on aggregates
 *     of consecutively numbered interface nodes form Shat = blkDiag(S_i)
 *     (section 3.1; Algorithm 1);
 *   - B = [D 0; F Shat][D^-1 0; 0 Shat^-1][D E; 0 Shat] (MSCN definition,
 *     section 3.3) is applied by Algorithm 2;
 *   - B is used as a right preconditioner of restarted GMRES (section 5 and
 *     the right-preconditioning remark of section 3.3).
 *
 * Conventions for every call:
 *   - indices are int32, values float64 at the boundary;
 *   - the caller owns every buffer it passes; the library owns its handles
 *     and the device memory behind them (freed by the *_destroy calls);
 *   - a call returns ADDNS_OK (0), a positive warning, or a negative error;
 *     addns_last_error() then holds a message for the calling thread.  No C++
 *     exception crosses this boundary;
 *   - "device" pointers are HIP device allocations on the current device;
 *     `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - a handle must not be used from two threads at once.
 */
#ifndef ADDNS_H
#define ADDNS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct addns_partition* addns_partition_t;
typedef struct addns_precond* addns_precond_t;

enum {
  ADDNS_OK = 0,
  ADDNS_WARN_SHARED_PAIR = 1, /* a closure node shares its paired interface node */
  ADDNS_ERR_ARG = -1,         /* invalid argument (message names it) */
  ADDNS_ERR_SINGULAR = -2,    /* zero/tiny pivot; message names the block */
  ADDNS_ERR_NOCONV = -3,      /* GMRES stopped at maxit above tol */
  ADDNS_ERR_HIP = -4,         /* a HIP runtime call failed */
  ADDNS_ERR_PARTITION = -5,   /* the graph could not be partitioned as asked */
  ADDNS_ERR_NOMEM = -6        /* host or device allocation failed */
};

/* Interface (Schur) approximation, Algorithm 1. */
enum {
  ADDNS_SCHUR_MSCN = 0,         /* S_i = G_i - F_i D_{r_i}^-1 E_i, D-range = interior
                                   velocity neighbours of the aggregate (section 3.1
                                   step 2b lets D_{r_i} exceed G_i in size) */
  ADDNS_SCHUR_MSCN_LITERAL = 1, /* D-range = the same positions of D (Algorithm 1) */
  ADDNS_SCHUR_LUM = 2,          /* S_i = G_i (LUM definition, section 3.3) */
  ADDNS_SCHUR_EXACT_BJ = 3,     /* diagonal blocks of the exact S = G - F D^-1 E */
  ADDNS_SCHUR_LEARNED = 4,      /* G_i plus a learned correction (opts.learned_model) */
  ADDNS_SCHUR_MSCNR = 5         /* rowsum variant (section 3.1 step 2; Algorithm 1):
                                   S_i = G_i - diag(F_i D_{r_i}^-1 E_i 1), MSCN's
                                   D-range; row sums of S_i equal MSCN's */
};

/* Storage precision of the preconditioner's factors (arithmetic is FP64 for
   the outer solver in every mode). */
enum { ADDNS_F64 = 0, ADDNS_F32 = 1, ADDNS_F16_SCALED = 2 };

/* ------------------------------------------------------------------------
 * addns_build_partition -- substructuring of C (section 1, the graph
 * partitioner paragraph; section 3.3).  Host-only integer work apart from
 * one exact-zero floating-point test; deterministic.
 *
 *   N, rowptr[N+1], colidx[nnz], vals[nnz]: HOST CSR of C (int32 / float64).
 *   m   : number of subdomains (>= 1), the nA of the paper's tables.
 *   sz  : aggregate size (>= 1), the paper's "sz" (MSC size).
 *   out : receives a new handle on success (unchanged on error).
 * The partition (recursive level-set bisection with a velocity-only
 * separator, closure of interior pressure components, reverse Cuthill-McKee
 * interior orderings, consecutive aggregates of size sz and their D-ranges)
 * keeps a copy of the pattern; the caller's arrays may be freed afterwards.
 * Returns ADDNS_OK, ADDNS_WARN_SHARED_PAIR, ADDNS_ERR_ARG or ADDNS_ERR_NOMEM.
 */
int addns_build_partition(int32_t N, const int32_t* rowptr, const int32_t* colidx,
                          const double* vals, int32_t m, int32_t sz, addns_partition_t* out);

/* Sizes of a partition: any pointer may be NULL. */
int addns_partition_info(addns_partition_t p, int32_t* N, int32_t* m, int32_t* n_interior,
                         int32_t* sep_size, int32_t* k, int32_t* drange_total);

/* ------------------------------------------------------------------------
 * addns_partition_export -- copy the partition into caller-owned HOST
 * arrays (any may be NULL):
 *   perm[N]           new position -> original index ([int_0..int_m-1, Sigma])
 *   part[N]           original index -> subdomain id, -1 = separator
 *   int_offsets[m+1]  offsets of the interiors in perm
 *   agg_offsets[k+1]  aggregate breakpoints r_i (0-based) in the separator order
 *   drange_offsets[k+1], drange_nodes[drange_total]: D-ranges (original indices)
 *   pair[sep_size]    per separator position: paired node (original) or -1
 */
int addns_partition_export(addns_partition_t p, int32_t* perm, int32_t* part,
                           int32_t* int_offsets, int32_t* agg_offsets, int32_t* drange_offsets,
                           int32_t* drange_nodes, int32_t* pair);

/* ------------------------------------------------------------------------
 * addns_partition_coarse_space -- the coarse space of the two-level
 * interface solve (opts.coarse = piece), copied into caller-owned HOST
 * arrays.  Section 6 proposes a coarse grid correction without fixing one;
 * this one is built from the pattern and the partition only:
 *   velocity classes = connected components of the pattern over the
 *   non-pressure nodes; two separator nodes of one class are near when they
 *   are coupled or share a coupled node; walking the separator in order, each
 *   velocity node not yet taken starts a piece that grows breadth first
 *   through near, free nodes (ascending positions) up to `piece` nodes; every
 *   piece gives a normalised constant column and, with >= 3 nodes, a
 *   normalised mean-free breadth-first level from the node last reached
 *   from its first node (ties: smaller position).
 *   piece  : P in 1..64 (else ADDNS_ERR_ARG).
 *   npieces, ncols: counts (either may be NULL); call once with NULL arrays
 *            to size them.
 *   piece_offsets[npieces+1], piece_pos[#velocity separator nodes]: members
 *            of each piece (separator positions, in joining order).
 *   col_piece[ncols], col_kind[ncols]: piece and kind (0 constant, 1 linear)
 *            of every column, in column order.
 *   z0[sep_size], z1[sep_size]: constant / linear value at each separator
 *            position (0 where none).
 * Host-only; deterministic.  Returns ADDNS_OK or ADDNS_ERR_ARG.
 */
int addns_partition_coarse_space(addns_partition_t p, int32_t piece, int32_t* npieces, int32_t* ncols,
                                 int32_t* piece_offsets, int32_t* piece_pos, int32_t* col_piece,
                                 int32_t* col_kind, double* z0, double* z1);

/* ------------------------------------------------------------------------
 * addns_partition_concat -- partition of the block-diagonal matrix
 * diag(C_0, ..., C_{nsys-1}) from the partitions of its independent blocks
 * (the batched form: every phase of setup and apply then runs as one launch
 * over the subdomains and aggregates of all systems).  Node s of system q is
 * node offset_q + s, offset_q = N_0 + ... + N_{q-1}; subdomains and
 * aggregates keep their system order; interiors of all systems come first
 * in perm, then all separators.  The inputs are not modified and stay owned
 * by the caller.  Returns ADDNS_OK, ADDNS_ERR_ARG or ADDNS_ERR_NOMEM.
 */
int addns_partition_concat(const addns_partition_t* parts, int32_t nsys, addns_partition_t* out);

typedef struct {
  int32_t schur;          /* ADDNS_SCHUR_* */
  int32_t interior_prec;  /* ADDNS_F64 or ADDNS_F32: storage of the A_jj factors */
  int32_t schur_prec;     /* ADDNS_F64, ADDNS_F32 or ADDNS_F16_SCALED: Shat^-1 */
  int32_t row_scale;      /* 1 = scale rows by their max |entry| (the paper's default) */
  const float* learned_model; /* LEARNED only: HOST array of addns_dtn_param_count()
                                  FP32 network weights (addns_dtn_train output) */
  int32_t block_mult;     /* interior sweep block size as a multiple of its minimum
                             (1..4); 0 = the library's fixed choice (1).  A tile
                             shape only: the factors are the same LU, regrouped;
                             results agree to rounding.  Whatever the value,
                             every setup times the sweep with and without
                             skipping the blocks' structural-zero row slots and
                             keeps the faster: the two forms give the same result
                             bit for bit, so this timing never changes numerics */
  int32_t learned_bf16;   /* LEARNED only: 1 = run the network with BF16-rounded
                             weights and activations, 0 = FP32 */
  int32_t overlap;        /* overlapped aggregates, w >= 0 (0 = none; the overlap
                             Remark of section 3.1 and Algorithm 1's overlapped
                             branch: OMSCN, OMSCNR, OLUM with schur = MSCN, MSCNR,
                             LUM; any other mode gives ADDNS_ERR_ARG).  Aggregate i
                             is extended by the first w_i = min(w, s_i - 1, s_{i+1})
                             separator positions of aggregate i+1 (w_k = 0); its
                             D-range is aggregate i's followed by aggregate i+1's.
                             The columns of each extended block S_i^e that belong
                             to aggregate i go, with all their rows, into Shat,
                             which becomes block lower bidiagonal; the interface
                             solve is then a forward substitution over the
                             aggregates (k - 1 dependent steps in one workgroup).
                             Needs every aggregate to hold at most 128 nodes
                             and at most 12000 aggregates (else ADDNS_ERR_ARG) */
  double ilu_tol;         /* 0: exact band LU of every interior block (section 4).
                             tau in (0, 1): threshold ILU, the inexact interior
                             solver of the experiments (section 5, tolerance 1e-4;
                             Algorithm 2 allows an inexact solve): during the
                             band elimination with partial pivoting, a multiplier
                             whose entry before division is below
                             tau ||A_jj(:,j)||_2 and a pivot-row entry u_jk below
                             tau ||A_jj(:,k)||_2 are dropped (column norms of the
                             scaled block before elimination); pivots are kept.
                             The sweep applies the incomplete factors exactly.
                             Outside [0, 1): ADDNS_ERR_ARG */
  int32_t sweep_chunks;   /* chunks p per subdomain of the interior sweep: the
                             lower and upper block recurrences of every interior
                             are cut at p - 1 upper-block boundaries, the chunks
                             are swept side by side from a zero incoming carry
                             (lower) or state (upper), and each chunk's result is
                             then corrected by its precomputed response to the
                             true carry or state, which a short recurrence over
                             the chunks supplies.  The same L and U factors and
                             the same solution, to rounding; more workgroups per
                             interior at the price of p - 1 small GEMVs on the
                             chunk boundaries and the response matrices' bytes.
                             0 = the p minimising a fixed cost model of the plan
                             (longest chunk's upper blocks at 17.5 us each plus
                             5 us per chunk boundary, at most one workgroup per
                             CU): no timing, so the same p, and the same
                             rounding, on every run; 1 = never;
                             p >= 2 = that many (ADDNS_ERR_ARG if an interior has
                             fewer than p upper blocks) */
  int32_t coarse;         /* coarse-grid correction of the interface solve (the
                             coarse grid correction section 6 proposes), 0 = none.
                             P in 1..64: the coarse space Z holds, for every
                             piece of at most P separator velocity nodes (grown
                             breadth first through nodes of one velocity class at
                             graph distance <= 2, see
                             addns_partition_coarse_space), a normalised constant
                             and a normalised linear coordinate; the interface
                             step of Algorithm 2 becomes
                               y = (Z^T S Z)^-1 Z^T t,
                               x2 = Z y + Shat^-1 (t - S Z y),
                             S = G - F D^-1 E formed on Z at setup from one
                             interior solve per (subdomain, coarse column) pair.
                             Theorem 2 holds with Shat^-1 replaced by this
                             operator.  At most 8192 coarse columns; not with
                             overlap > 0 (else ADDNS_ERR_ARG); a singular
                             Z^T S Z gives ADDNS_ERR_SINGULAR.  (Z^T S Z)^-1 is
                             formed by Gauss-Jordan elimination in one of four
                             kernel forms that give the same inverse bit for
                             bit; the environment variable ADDNS_COARSE_GJ
                             (lds, registers, memory, steps) forces one, for
                             tests: a form too small for the coarse blocks gives
                             ADDNS_ERR_ARG */
  int32_t sweep_zero_skip;  /* sweep form: 0 = time the sweep with and without
                             loading only each stored column's nonzero rows and
                             keep the faster (the default; both give the same
                             result bit for bit; a later setup on the same
                             partition and device with the same interior_prec,
                             sweep_chunks and ilu_tol reuses the first timing);
                             1 = never skip; 2 = always skip; else
                             ADDNS_ERR_ARG */
  int32_t block_sizing;   /* sweep block sizes: 1 = one size for every interior
                             (the widest band sets it: fewest dependent steps);
                             2 = each interior its own (fewest bytes and least
                             work); 0 = 2 when the interiors outnumber the
                             device's compute units (their workgroups then queue
                             and the total work counts), else 1: a rule of the
                             plan and the device, no timing.  The two regroup
                             the same factors into different blocks, so their
                             solves agree to rounding only; else ADDNS_ERR_ARG */
  int32_t overlap_segment; /* overlap > 0: the forward substitution over the
                             aggregates, x_i = u_i - M_i x_{i-1}, runs in
                             segments of L aggregates: each segment from a zero
                             start side by side, a chain over the segments'
                             last aggregates with the responses
                             Q_i = -M_i Q_{i-1} (Q = M at a segment's first
                             aggregate, formed at setup), and x_i = z_i -
                             Q_i x_(previous segment's last) for the rest.  The
                             same Shat^-1, to rounding.  0 = L = ceil(sqrt(k))
                             (the default); L >= k = one chain; < 0:
                             ADDNS_ERR_ARG */
} addns_precond_opts;

/* ------------------------------------------------------------------------
 * addns_setup_precond -- Algorithm 1 plus the exact interior factorisations
 * ([L,U] = lu(A_jj), section 4).  All floating-point work runs on the GPU.
 *
 *   p      : partition built from the same pattern (rowptr/colidx equal).
 *   N, d_rowptr, d_colidx, d_vals: DEVICE CSR of C (unscaled); read during
 *            the call only.
 *   opts   : NULL = MSCN, FP64 factors, row scaling on.
 *   stream : hipStream_t as void*; the call returns after the setup work has
 *            completed on that stream.
 *   out    : receives a new handle.  The handle owns a scaled, permuted copy
 *            of C and all factors.
 * Errors: ADDNS_ERR_ARG (size mismatch), ADDNS_ERR_SINGULAR (an interior or
 * interface block has a zero pivot; message names it), ADDNS_ERR_HIP,
 * ADDNS_ERR_NOMEM.
 */
int addns_setup_precond(addns_partition_t p, int32_t N, const int32_t* d_rowptr,
                        const int32_t* d_colidx, const double* d_vals,
                        const addns_precond_opts* opts, void* stream, addns_precond_t* out);

/* ------------------------------------------------------------------------
 * addns_precond_refactor -- new values on the same sparsity pattern, as in
 * an outer Picard iteration (section 1: every outer step is an Oseen system
 * whose wind is the previous velocity).  Every numeric part of
 * addns_setup_precond is recomputed for d_vals (row scaling, interior band
 * LU and sweep blocks, mini Schur complements, inverses, chain matrices),
 * keeping the handle's partition plan, options, sweep block size and
 * zero-slot choice: no host planning and no autotuning.  Device buffers
 * keep their sizes and addresses, so an apply captured in a HIP graph
 * before the call uses the new factors when replayed after it.
 *   d_rowptr, d_colidx: DEVICE CSR pattern, identical to the setup's (not
 *            checked); d_vals: DEVICE values of C (unscaled).
 * Returns after the work has completed on `stream`.  Errors as
 * addns_setup_precond; after a failed refactor the handle holds no factors
 * (apply, solve and block queries return ADDNS_ERR_ARG) until a refactor
 * succeeds.
 */
int addns_precond_refactor(addns_precond_t pc, const int32_t* d_rowptr, const int32_t* d_colidx,
                           const double* d_vals, void* stream);

/* ------------------------------------------------------------------------
 * addns_apply_precond -- Algorithm 2: x = B^{-1} y,
 *   z1 = D^-1 y1;  x2 = Shat^-1 (y2 - F z1);  x1 = z1 - D^-1 (E x2),
 * for DEVICE vectors of length N in the ORIGINAL numbering of the scaled
 * system (y, x must not alias).  Asynchronous on `stream`.  It only launches
 * kernels (no allocation, copy, memset or synchronisation), so a caller can
 * capture it in a HIP graph and replay it; it works in the handle's own
 * permuted vectors, so applies on one handle must not overlap.
 */
int addns_apply_precond(addns_precond_t pc, const double* d_y, double* d_x, void* stream);

/* ------------------------------------------------------------------------
 * addns_apply_precond_static -- addns_apply_precond for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and the same result bit
 * for bit, with the permuted in/out vectors and the interior sweeps' padded
 * work vectors in a library-static device array instead of the handle's.
 * The call allocates and frees nothing.
 *   pc, d_y, d_x, stream: as for addns_apply_precond (d_x must not alias d_y).
 * Limit: the array holds 4 Mi doubles (32 MiB); a system needing more than
 * 2 N + 2 (padded interior rows) doubles gives ADDNS_ERR_ARG, as does a
 * current device other than the handle's.  Every GPU holds one copy of the
 * array until the process ends, shared by all calls on that GPU: calls on
 * one GPU whose execution overlaps (different streams, threads or handles)
 * race on it and must be serialised by the caller.  Nothing in the array
 * needs to start at zero (every entry read is first written by the call).
 */
int addns_apply_precond_static(addns_precond_t pc, const double* d_y, double* d_x, void* stream);

/* ------------------------------------------------------------------------
 * addns_interior_solve -- the interior block solve of Algorithm 2 on its
 * own: z1 = D^{-1} y1 with D = blkDiag(A_11..A_mm), for DEVICE vectors of
 * length n_interior in the PERMUTED interior order (perm[0..n_interior) of
 * addns_partition_export).  y1 and z1 must not alias.  Asynchronous on
 * `stream`.  Runs the same kernel as the two interior sweeps of
 * addns_apply_precond.
 */
int addns_interior_solve(addns_precond_t pc, const double* d_y1, double* d_z1, void* stream);

typedef struct {
  int32_t restart;   /* Krylov dimension per cycle (1..1024) */
  int32_t maxit;     /* total inner iterations allowed */
  double tol;        /* stop when ||b~ - C~ x|| / ||b~|| <= tol */
  int32_t flexible;  /* 1 = FGMRES (store Z), 0 = GMRES (x += B^-1 V y) */
  int32_t use_x0;    /* 1 = d_x holds the initial guess, 0 = start from zero */
  int32_t ortho;     /* Arnoldi orthogonalisation (section 5 leaves it open):
                        ADDNS_ORTHO_MGS, modified Gram-Schmidt, one launch per
                        basis vector; ADDNS_ORTHO_CGS2, classical Gram-Schmidt
                        applied twice, all inner products of a pass in one
                        launch (5 launches per iteration whatever the basis
                        size).  The batched solver takes MGS only. */
} addns_gmres_opts;

enum { ADDNS_ORTHO_MGS = 0, ADDNS_ORTHO_CGS2 = 1 };

typedef struct {
  int32_t iters;         /* inner iterations taken */
  int32_t cycles;        /* restart cycles */
  int32_t converged;     /* 1 if the true relative residual <= tol */
  double true_relres;    /* ||b~ - C~ x|| / ||b~|| of the returned x (scaled system) */
  double est_relres;     /* |g_{j+1}| / ||b~|| at the last iteration */
  double* resid_hist;    /* optional HOST array of maxit+1 entries (may be NULL):
                            estimated relative residual after each iteration */
} addns_gmres_result;

/* ------------------------------------------------------------------------
 * addns_gmres_solve -- restarted (F)GMRES with right preconditioning by B,
 * Arnoldi by modified or twice-applied classical Gram-Schmidt (opts.ortho)
 * and Givens rotations, all in FP64 on the
 * GPU (section 5 accelerator).  Solves C x = b through the row-scaled system.
 *   d_b : DEVICE right-hand side of the unscaled system (length N).
 *   d_x : DEVICE solution (length N); initial guess if opts.use_x0.
 * Returns after completion.  ADDNS_ERR_NOCONV when maxit is reached above
 * tol (x then holds the last iterate and res the true residual).
 */
int addns_gmres_solve(addns_precond_t pc, const double* d_b, double* d_x,
                      const addns_gmres_opts* opts, addns_gmres_result* res, void* stream);

/* ------------------------------------------------------------------------
 * addns_precond_fill -- the fill factor of section 5 (the preconditioner's
 * nonzeros over those of C): *nnz_precond = the nonzero entries of the
 * interior factors L_j (multipliers) and U_j (with the diagonal), the
 * entries of the interface blocks S_i (dense, s_i^2 each; with overlapped
 * aggregates also the lower blocks of Shat), and the entries of E and F that
 * Algorithm 2 applies; *nnz_c = nnz(C).  The coarse correction is not
 * counted.  Either pointer may be NULL.  Returns ADDNS_OK or ADDNS_ERR_ARG.
 */
int addns_precond_fill(addns_precond_t pc, int64_t* nnz_precond, int64_t* nnz_c);

/* ------------------------------------------------------------------------
 * addns_gmres_solve_batched -- one independent restarted FGMRES per system
 * of a block-diagonal matrix (preconditioner built on an
 * addns_partition_concat partition), all systems advanced in lockstep:
 * every kernel launch serves all systems still iterating; each system has its
 * own Krylov basis segment, Hessenberg matrix, rotations, stopping test and
 * iteration count, and stops (is frozen) on its own.  Mathematically each
 * system follows addns_gmres_solve with opts.flexible = 1.
 *   sys_offsets : HOST, nsys+1 increasing row offsets of the systems in the
 *                 original numbering (0 .. N).
 *   d_b, d_x    : DEVICE, length N (x: initial guess if opts.use_x0).
 *   res         : HOST array of nsys results (resid_hist pointers optional).
 * Returns ADDNS_ERR_NOCONV if any system stops at maxit above tol.
 */
int addns_gmres_solve_batched(addns_precond_t pc, int32_t nsys, const int32_t* sys_offsets,
                              const double* d_b, double* d_x, const addns_gmres_opts* opts,
                              addns_gmres_result* res, void* stream);

/* Sizes of a preconditioner: any pointer may be NULL.  bytes_apply is the
   algorithmic byte count of one apply (band factors read once per sweep,
   pivots, coupling blocks, interface inverses, vector passes); block_mult
   is the sweep tile multiplier in use (0 in the options is taken as 1);
   learned_count is the number of learned-correction
   samples (separator velocity rows); interior_nnz is the number of stored
   entries of the interior factors (multipliers below the unit diagonal and
   U, real rows and columns), the numerator of the fill factor of section 5
   with or without ILU dropping; sweep_chunks is the chunk count p of the
   interior sweep in use (1 = one workgroup per interior) and chunk_bytes the
   size of its response matrices, read once per interior solve (included
   twice in bytes_apply).  kl and ku are the largest band widths over the
   interiors; band_words is sum_j n_j (2 kl_j + ku_j + 1), the entries of the
   interior band factors with each interior's own widths (the factors one
   interior solve reads, section 4, Algorithm 2). */
int addns_precond_info(addns_precond_t pc, int32_t* kl, int32_t* ku, int32_t* nb_lower,
                       int32_t* nb_upper, int64_t* factor_bytes, int64_t* bytes_apply,
                       int64_t* learned_count, int32_t* block_mult, int64_t* interior_nnz,
                       int32_t* sweep_chunks, int64_t* chunk_bytes, int64_t* band_words);

/* Copy the dense interface blocks S_i (before inversion) into a HOST array
   in aggregate order, row-major per block; `count` must equal the sum of
   |agg_i|^2.  With overlapped aggregates these are the extended blocks
   S_i^e, (s_i + w_i)^2 numbers each. */
int addns_precond_schur_blocks(addns_precond_t pc, double* h_out, int64_t count);

/* ========================================================================
 * Learned interface correction -- an extension, not a method of the paper.
 * The exact interface Schur complement S = G - F D^-1 E (section 1; the
 * algebraic Dirichlet-to-Neumann map) is approximated blockwise by the MSCN
 * blocks of section 3.1: exact Schur complements of the local systems on
 * the aggregates' D-ranges.  Here a small network predicts, for each
 * separator velocity row, corrections on G's own stencil pattern,
 *   S_i ~ G_i + Delta_i,
 * trained on the blocks of a teacher mode (MSCN by default; EXACT_BJ, the
 * diagonal blocks of the exact S, is also available):
 *   features (7, FP32): the five scaled stencil coefficients of the row in
 *     the slots [far lower, near lower, diagonal, near upper, far upper]
 *     (neighbours ordered by distance in the original numbering, velocity
 *     unknowns only) and the skew (convective) differences near and far;
 *   network: 7 -> 64 -> 64 -> 5, ReLU, row-major W1[64][7] b1[64] W2[64][64]
 *     b2[64] W3[5][64] b3[5];
 *   targets: S_i - G_i on the slots whose neighbour lies in the same
 *     aggregate (mask 1), else 0 (mask 0); loss (1/count) sum mask (p - y)^2.
 * The learned blocks are sparse where the teacher's are dense, so solves
 * with them go through addns_gmres_solve_judged, which accepts them only
 * when the FP64 true residual reaches the tolerance.
 * ====================================================================== */

/* Number of FP32 network parameters (4997). */
int addns_dtn_param_count(void);

/* Training samples of a preconditioner (the teacher: any mode except
   LEARNED), one per separator velocity row, into DEVICE arrays X[count][7]
   and, optionally together, Y[count][5] and M[count][5] (FP32); the
   targets are S_i - G_i of the teacher's interface blocks.  With all three
   NULL only *count is set (a size query).  cap: capacity in samples.
   Asynchronous on `stream`.  ADDNS_ERR_ARG for a LEARNED handle, Y without
   M (or M without Y), targets of a handle with overlapped aggregates, or
   cap < count. */
int addns_dtn_samples(addns_precond_t pc, float* d_X, float* d_Y, float* d_M, int64_t cap,
                      int64_t* count, void* stream);

/* Network output P[count][5] for DEVICE features X[count][7]; weights on the
   HOST (param_count FP32).  bf16 = 1 rounds weights, inputs and hidden
   activations to BF16 (round to nearest even), accumulating in FP32.
   Returns after completion. */
int addns_dtn_forward(const float* h_weights, const float* d_X, float* d_P, int64_t count,
                      int32_t bf16, void* stream);

/* Full-batch gradient of the loss in FP32 (fixed reduction order) into the
   HOST array h_grad[param_count]; *loss receives the loss (may be NULL).
   Returns after completion. */
int addns_dtn_grad(const float* h_weights, const float* d_X, const float* d_Y, const float* d_M,
                   int64_t count, float* h_grad, double* loss, void* stream);

typedef struct {
  int32_t epochs;     /* passes over the samples (>= 0) */
  int32_t batch;      /* minibatch size (>= 1) */
  float lr;           /* Adam step size (> 0) */
  float beta1, beta2, eps; /* Adam moments and guard */
  int64_t seed;       /* initialisation and shuffling (host mt19937_64) */
  int32_t init_given; /* 1 = start from h_weights, 0 = seeded He-uniform init */
} addns_dtn_params;

/* Minibatch Adam training on the GPU in FP32 over DEVICE samples.  The
   weights are returned in h_weights (HOST, param_count).  h_loss (HOST,
   epochs entries, may be NULL) receives the full-data loss after each
   epoch.  Deterministic for a given seed.  Returns after completion. */
int addns_dtn_train(const float* d_X, const float* d_Y, const float* d_M, int64_t count,
                    const addns_dtn_params* hp, float* h_weights, double* h_loss, void* stream);

/* Weights file: 8-byte tag "ADDNSDTN", int32 parameter count, FP32 weights
   (little endian).  ADDNS_ERR_ARG on a missing file, a wrong tag or count. */
int addns_dtn_save(const char* path, const float* h_weights);
int addns_dtn_load(const char* path, float* h_weights);

/* Judged solve: addns_gmres_solve with `learned`; if it does not reach
   opts.tol in FP64 true relative residual within opts.maxit, the same solve
   is run again with `plain` from the caller's initial guess.  *accepted = 1
   when the learned result was kept.  The two handles must be set up on the
   same matrix. */
int addns_gmres_solve_judged(addns_precond_t learned, addns_precond_t plain, const double* d_b,
                             double* d_x, const addns_gmres_opts* opts, addns_gmres_result* res,
                             int32_t* accepted, void* stream);

/* A partition keeps the host plans of its setups and, after a first setup on
   a device, that setup's index maps on the device (gathers and scatters of
   the matrix entries, about 16 bytes per nonzero), so that a repeated setup
   of the same partition uploads none of them; destroying the partition
   releases both. */
void addns_partition_destroy(addns_partition_t p);
void addns_precond_destroy(addns_precond_t pc);

/* Device memory of the library.  Every device buffer that a handle or a call
   owns comes from a per-device cache: a released buffer is kept, not freed,
   and is handed out again (for a request of at most its size and at least
   half of it) once a device synchronisation has followed its release (each
   addns_setup_precond begins with one when there are released buffers), so
   repeated setups and solves do not pay hipMalloc/hipFree, which also
   synchronises the device, per buffer.  At most a quarter of the device
   memory is kept; beyond that a release frees at once.  This call
   synchronises every device that holds cached buffers, frees them all and
   returns the number of bytes freed (0 if none).  Buffers of live handles
   are not touched.  No stream argument: it waits for all work on the device. */
int64_t addns_release_cached_memory(void);

/* Message of the last error on the calling thread ("" if none). */
const char* addns_last_error(void);

/* Library version string. */
const char* addns_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ADDNS_H */
