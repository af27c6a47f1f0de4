/*
 * thc.h -- C ABI of the MI355X (gfx950) THC-CCSD hot path.
 *
 * Method: tensor-hypercontracted rank-reduced CCSD (Hohenstein, Fales, Parrish, Martinez,
 * "Rank-reduced coupled-cluster III", arXiv:2111.11473).  The doubles amplitudes are
 *   t_ij^ab = sum_WX y_i^W y_a^W Z^WX y_j^X y_b^X                         (paper Eq. 22-23)
 * and the unknown core Z solves the projected CCSD doubles equations
 *   sigma^WX = sum_ijab y_i^W y_a^W <Phi_ij^ab| e^-T H e^T |0> y_j^X y_b^X = 0   (Eq. 6),
 * together with the usual singles equations, with the T1-transformed Hamiltonian (Eq. 24-27),
 * Cholesky integrals (pq|rs) = sum_A L_pq^A L_rs^A and the least-squares THC form of (ia|jb)
 * (Eq. 17-20) in the quadratic terms.
 *
 * Conventions
 *  - Every array argument is a DEVICE pointer (memory on the GPU the context was created on),
 *    row-major, FP64 (FP32 where the declaration takes float), owned by the caller; the library
 *    copies what it keeps.  The few host arrays are marked HOST or "host" at their declaration.
 *    Scalars returned through pointers (energies, norms, iteration counts) are HOST pointers.
 *  - Sizes: o occupied, v virtual, n = o + v orbitals, nL Cholesky vectors, nP amplitude THC
 *    rank, nQ ERI THC grid points.
 *  - All work is issued on the stream given to thc_create (a hipStream_t, e.g. torch's current
 *    stream); functions that return host scalars synchronize that stream.
 *  - Return value: THC_OK (0) or a negative error code; thc_last_error() gives a message.
 *    No C++ exception crosses the ABI.  One context must not be used by two threads at once.
 */
#ifndef THC_H
#define THC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define THC_OK 0
#define THC_EINVAL (-1)     /* bad argument or option */
#define THC_ENOMEM (-2)     /* device allocation failed */
#define THC_EDEVICE (-3)    /* HIP runtime error */
#define THC_ESINGULAR (-4)  /* metric S or ERI-grid Gram matrix not positive definite */
#define THC_ENUMERIC (-5)   /* NaN/Inf in a residual or energy */
#define THC_ENOTCONV (-6)   /* iteration limit reached */
#define THC_ESTATE (-7)     /* call out of order (e.g. residual before build_factors) */
#define THC_EDIVERGED (-8)  /* thc_iterate diverged, restarted from the MP2 guess, and diverged again */

/* Residual term groups (bit mask for thc_residual_terms), named by the paper's equations. */
#define THC_TERM_EQ28 (1u << 0)   /* pp/hh/mixed ladders, Alg. 1 */
#define THC_TERM_EQ29 (1u << 1)   /* bare integrals + Coulomb rings, Alg. 2 */
#define THC_TERM_EQ31 (1u << 2)   /* remaining linear terms, Alg. 3 */
#define THC_TERM_EQ32 (1u << 3)   /* T2^2 ladder + exchange (Eq. 32 + 33), Alg. 6 */
#define THC_TERM_EQ35 (1u << 4)   /* T2^2 rings (Eq. 35-37), Alg. 7 */
#define THC_TERM_EQ41 (1u << 5)   /* Fock + xi intermediates, Alg. 8-9 */
#define THC_TERM_EQ38 (1u << 6)   /* singles, Alg. 8 */
#define THC_TERM_EQ42 (1u << 7)   /* singles Fock terms, Alg. 10 */
#define THC_TERM_ALL 0xffu

typedef struct thc_ctx thc_ctx;

typedef struct thc_options {
  int64_t o, v, nL, nP, nQ; /* problem sizes (all >= 1) */
  int32_t singles;          /* 1: CCSD (T1-dressed), 0: CCD (t1 fixed at zero) */
  int32_t diis_max;         /* DIIS subspace size; 0 disables DIIS (<= 16) */
  double tol_energy;        /* |dE| convergence threshold (Eh), e.g. 1e-8 */
  int64_t a_block;          /* Cholesky vectors per fused-pass block; 0 = automatic */
  int64_t i_chunk;          /* ERI grid points per H-kernel pass; 0 = automatic */
  int64_t x_block;          /* amplitude ranks per H block (multiple of 64, at most nP rounded up to 64);
                             * 0 = automatic */
  int64_t x_chunk;          /* amplitude ranks per Alg. 7 exchange chunk (two-GEMM form); 0 = automatic */
  int32_t precision;        /* 0 = FP64 throughout; 1 = mixed: FP32-MFMA contractions (the fused Alg. 7
                               exchange included) and the H accumulation in FP32 per grid-point chunk
                               (added into an FP64 H),
                               FP64 energy, denominators, fit and DIIS, and thc_iterate finishing with
                               FP64 residuals (mixed ones until the norm has dropped 1e4-fold, is
                               within 10 tol, stops falling, or the last two predict the next one
                               below tol; only an FP64 residual declares convergence); 2 = as 1 with the GEMM contractions as compensated
                               split-BF16 products (each FP32-rounded operand split exactly into
                               three bf16 pieces, the six largest cross products on BF16 MFMA,
                               FP32 accumulation); the fused exchange stays FP32 MFMA */
  int32_t flags;            /* THC_FLAG_* bits; 0 = defaults */
  int64_t x7_chunk;         /* amplitude ranks X per chunk of the Alg. 7 intermediates (R^X, S^X
                             * half-transformed, exchange outputs); 0 = automatic */
  int64_t q_pairs;          /* Alg. 4 and 5: pairs per batched product; 0 = automatic */
  int64_t q_jchunk;         /* Alg. 4 and 5: occupied j per chunk of the dense residual; 0 = automatic */
  uint64_t split_mask;      /* precision 1 only: THC_CHAIN_* bits of the contraction chains whose GEMMs
                               run as compensated split-BF16 products instead of FP32 MFMA
                               (precision 2 is every chain); 0 = none */
  int32_t guess;            /* starting point of the first thc_iterate after thc_build_factors:
                               0 = the MP2 guess; 1 = the learned guess of the network given to
                               thc_set_guess_network (falls back to the MP2 guess with the plain
                               denominators if the iteration diverges from it, or has not cut the
                               residual norm tenfold after three iterations) */
  int32_t reserved;         /* 0 */
} thc_options;

/* Contraction chains of the residual (bits of thc_options.split_mask). */
#define THC_CHAIN_FUSED (1u << 0)    /* fused pass over Cholesky vectors: Alg. 1 panels and core, Alg. 2, 3, 8 */
#define THC_CHAIN_ASSEMBLY (1u << 1) /* assembly of the symmetric terms: Alg. 2, 3, 9 */
#define THC_CHAIN_ALG45 (1u << 2)    /* Alg. 4 and 5 (when the cost model takes them) */
#define THC_CHAIN_ALG6 (1u << 3)     /* the matrix products of Alg. 6 around the H accumulation */
#define THC_CHAIN_ALG7 (1u << 4)     /* Alg. 7 (its fused exchange kernel stays FP32 MFMA) */
#define THC_CHAIN_SINGLES (1u << 5)  /* singles residual: Alg. 8 and 10 */
#define THC_CHAIN_ALL 0x3Fu

/* Alg. 7 exchange contraction: by default fused on chip (no Q x Q intermediate) when o <= 200;
 * this flag forces the two-GEMM form with its x_chunk-blocked Q x Q intermediate instead. */
#define THC_FLAG_UNFUSED_EXCHANGE (1 << 0)
/* Synthetic inputs only (thc_set_synthetic): the vv block of the Cholesky vectors is not held in
 * device memory but regenerated for each block of the fused pass over Cholesky vectors (the
 * default when it does not fit the memory plan). */
#define THC_FLAG_STREAM_LVV (1 << 1)
/* Print a line to stderr after each block of the residual's outer loops (fused pass over
 * Cholesky vectors, Alg. 6 H blocks, Alg. 7 row chunks), waiting for the stream each time. */
#define THC_FLAG_PROGRESS (1 << 2)
/* The quadratic ladder and exchange terms (Eq. 32 + 33): by default the context takes whichever of
 * the paper's two algorithms its cost model estimates faster -- Alg. 4 and 5 (O(N^5), every step
 * a matrix product; small systems) or Alg. 6 (O(N^4) with the three-way H accumulation).  These
 * flags force one (not both). */
#define THC_FLAG_QUINTIC (1 << 3)
#define THC_FLAG_QUARTIC (1 << 4)
/* Debugging: wait for the stream after every device step of the context, so that a device error
 * is returned (THC_EDEVICE, thc_last_error naming the step) by the step that caused it. */
#define THC_FLAG_CHECK (1 << 5)

/* Creates a context bound to the current HIP device and to `stream` (hipStream_t; NULL = the
 * default stream).  Allocates nothing on the device yet.  *out receives the context.
 * THC_EINVAL for sizes below 1, nP or nQ above o v (the metric of the pair basis and the Gram
 * matrix of the ERI grid would be singular), or options out of range; nothing is created then. */
int thc_create(const thc_options* opt, void* stream, thc_ctx** out);

/* As thc_create, with all device working memory taken from the caller's workspace: the library
 * then never allocates device memory (set-up scratch included).  dev_workspace: device pointer,
 * 256-byte aligned, ws_bytes long, owned by the caller and kept alive until thc_destroy.  The
 * plan (blocking of the paper's loops) is sized to ws_bytes; thc_plan_query gives the bytes a
 * plan needs.  THC_ENOMEM from thc_build_factors if no plan fits. */
int thc_create_with_workspace(const thc_options* opt, void* dev_workspace, size_t ws_bytes, void* stream,
                              thc_ctx** out);

/* Set-up (paper Eq. 9-14, 17-20; Alg. 6): copies the integrals and factors, forms the
 * Gram matrices o = Xo^T Xo, v = Xv^T Xv and the metric S = o (Hadamard) v, fits the ERI core
 * z = xi^T xi by least squares against the ovov Cholesky block, forms B_ia^I, solves the
 * generalized eigenproblem of the projected Fock operator (E w = e S w, the working basis with
 * exact denominators e_P + e_Q) and the least-squares fit of the MP2 amplitudes,
 * Z0 = S^-1 B^T t_MP2 B S^-1, which becomes the current state (t1 = 0).
 *   L   [nL][n][n]  Cholesky vectors in the MO basis, symmetric in (p, q), occupied first
 *   eps [n]         orbital energies (the Fock matrix is diag(eps))
 *   X   [o*nP + v*nP + o*nQ + v*nQ]  Xo[o][nP] | Xv[v][nP] | xo[o][nQ] | xv[v][nQ]
 *   Z   [nP][nP]    out: the MP2-guess core (may be NULL)
 * L, eps and X are NULL after thc_set_synthetic (the inputs are generated on the device).
 * Allocates the device working memory (all of it; nothing is allocated later). */
int thc_build_factors(thc_ctx* ctx, const double* L, const double* eps, const double* X, double* Z);

/* Seeded synthetic inputs generated on the device instead of caller arrays (the workloads'
 * stand-in for molecules): eps_o ~ U[-1.5, -0.3], eps_v ~ U[0.1, 5.0] (each sorted ascending),
 * L^K_pq = gamma N(0,1) e^(-K/decay) symmetric in (p, q), Xo, Xv ~ N(0,1)/sqrt(nP),
 * xo, xv ~ N(0,1)/sqrt(nQ), from counter-based SplitMix64 draws (Steele, Lea & Flood 2014) with
 * Box-Muller normals; stream s of seed S gives the same values, bit for bit, as the Python
 * generator of the package (streams: 0 eps_o, 1 eps_v, 2 L (draw K n^2 + p n + q, p <= q),
 * 3 Xo, 4 Xv, 5 xo, 6 xv; all row-major).  gamma > 0 is used as given; otherwise it is fixed by
 * gamma^2 lambda_max(L_ov L_ov^T) = coupling (2 (eps_LUMO - eps_HOMO)), lambda_max by 200 steps
 * of power iteration on the nL x nL Gram matrix of the unscaled ov block from the normalized
 * all-ones vector.  Call before thc_build_factors, which then takes NULL for L, eps and X. */
typedef struct thc_synth_spec {
  uint64_t seed;
  double decay;    /* decay length of the Cholesky vectors (> 0) */
  double coupling; /* the gamma rule's fraction of the smallest pair gap (> 0 when gamma <= 0) */
  double gamma;    /* > 0: this scale; <= 0: the rule */
} thc_synth_spec;
int thc_set_synthetic(thc_ctx* ctx, const thc_synth_spec* spec);
/* The global scale gamma of the synthetic Cholesky vectors (host), valid after thc_build_factors. */
int thc_synth_gamma(const thc_ctx* ctx, double* gamma);

/* The generator itself, for callers that want the same inputs in their own buffers (device
 * arrays; work on `stream`).  thc_synth_normals: out[i] = (N(0,1) draw first + i of
 * (seed, stream_id)) / divisor, i < count.  thc_synth_cholesky: vectors K0 .. K0 + nK - 1 as
 * whole n x n matrices, L[nK][n][n], times gamma.  thc_synth_energies: eps[o + v] (HOST array). */
int thc_synth_normals(uint64_t seed, int32_t stream_id, uint64_t first, int64_t count, double divisor, double* out,
                      void* stream);
int thc_synth_cholesky(uint64_t seed, int64_t n, int64_t K0, int64_t nK, double decay, double gamma, double* L,
                       void* stream);
int thc_synth_energies(uint64_t seed, int64_t o, int64_t v, double* eps);

/* Residual of a state (pure: the context state is not changed).
 *   Z      [nP][nP] amplitude core (symmetric), raw collocation basis
 *   t1     [o][v]   singles (NULL = zero; ignored in CCD mode)
 *   sigma  [nP][nP] out: projected doubles residual sigma^WX (Eq. 6)
 *   sigma1 [o][v]   out: singles residual (may be NULL)
 *   norms  host [2] out: ||W^T sigma W||_F in the orthonormal working basis and ||sigma1||_F
 *                   (may be NULL; if given the call synchronizes the stream) */
int thc_residual(thc_ctx* ctx, const double* Z, const double* t1, double* sigma, double* sigma1, double* norms);

/* As thc_residual, restricted to the term groups in `mask` (THC_TERM_*). */
int thc_residual_terms(thc_ctx* ctx, const double* Z, const double* t1, uint32_t mask, double* sigma,
                       double* sigma1);

/* MP2 one-particle density matrix (unrelaxed, closed shell; paper App. II, Eq. 47-48) of the
 * amplitudes t = sum y y Z y y of a core, evaluated in O(N^4) through the Gram matrices o, v
 * (Eq. 51-56): D_ij = -2 sum_kab t_ik^ab (2 t_jk^ab - t_jk^ba), D_ab = 2 sum_ijc t_ij^ac
 * (2 t_ij^bc - t_ji^bc).  Z [nP][nP] raw basis (NULL: the current state, after thc_build_factors
 * the MP2 guess); Doo [o][o], Dvv [v][v] device outputs.  FP64. */
int thc_mp2_density(thc_ctx* ctx, const double* Z, double* Doo, double* Dvv);

/* Weighted CANDECOMP/PARAFAC of a 3-index array by alternating least squares (paper Sec. II.c
 * Eq. 15-16 and Sec. II.d Eq. 21: the factorization that turns the projectors and the Cholesky
 * vectors into THC form; Appendix I Eq. 43-46: its row-wise normal equations, solved by conjugate
 * gradients preconditioned with diag(S)).  Minimizes
 *     O = sum_ijk (w1_i w2_j w3_k)^2 (A_ijk - sum_n X_in Y_jn Z_kn)^2
 * by `sweeps` sweeps, each the update of X, then Y, then Z with the other two fixed.
 *   A          device [I][J][K]
 *   w1, w2, w3 device [I], [J], [K] weights (NULL: all ones)
 *   X, Y, Z    device [I][n], [J][n], [K][n]; in: the start, out: the factors after the sweeps
 *   cg_tol     each column's residual norm relative to its right-hand side ends the CG solve
 *   cg_maxit   iteration limit of one CG solve
 *   objective  HOST [sweeps + 1] out: O before the first sweep and after each (NULL: not computed)
 *   cg_iters   HOST out: the most CG iterations one solve took (may be NULL)
 * Work on `stream`; synchronizes it before returning.  Allocates and frees its own workspace
 * (about (IJ + 3 max(I, J, K) + 7 n) n doubles): it is a set-up step, not part of an iteration.
 * Returns THC_ENOTCONV if some solve reached cg_maxit (the factors are then still updated with the
 * last iterate), THC_EINVAL for bad sizes, THC_ENOMEM, THC_EDEVICE. */
int thc_cp_als(const double* A, int64_t I, int64_t J, int64_t K, int64_t n, const double* w1, const double* w2,
               const double* w3, double* X, double* Y, double* Z, int sweeps, double cg_tol, int cg_maxit,
               double* objective, int* cg_iters, void* stream);

/* Jacobi + DIIS iterations from the current state (the paper gives no update rule: this is the
 * standard denominator-weighted update in the working basis where the Fock part of the projected
 * residual is exactly diagonal, Sec. II's equations; Pulay DIIS): each iteration evaluates the
 * residual and the energy of the current amplitudes, stops when the residual norm (orthonormal
 * basis) is below tol and |dE| < tol_energy, else updates T^ -= sigma^/(e_P + e_Q),
 * t1 -= sigma1/(eps_a - eps_i) and extrapolates with DIIS (the oldest vectors dropped while the
 * error overlap matrix has a condition number above 1e12).  Divergence -- a residual norm or
 * energy that is not finite, a norm above 10 times the smallest of the call, or three rises in a
 * row -- restarts once from the MP2 guess with the plain denominators and an empty DIIS subspace
 * (within the same maxit); so does a learned start (thc_options.guess = 1) whose residual norm has
 * not fallen tenfold after three iterations.  *iters (host, may be NULL): residual evaluations; *rnorm (host, may be
 * NULL): last residual norm.  Returns THC_ENOTCONV when maxit is reached, THC_EDIVERGED when the
 * restarted iteration diverges too. */
int thc_iterate(thc_ctx* ctx, double tol, int maxit, int* iters, double* rnorm);
/* A call continues the previous call's iteration: its first |dE| test compares with the last
 * energy of that call, unless the state was set since (thc_build_factors, thc_set_state,
 * thc_guess_apply, thc_set_shift, thc_load_checkpoint with a fresh checkpoint). */

/* Solver checkpoint, for resuming an interrupted solve in another context (or process) built on
 * the same inputs and options: the state T^ (working basis) and t1, the denominator shift, the DIIS
 * subspace (vectors, errors, overlap matrix, position) and the last energy.  thc_checkpoint_bytes
 * gives the size, (P^2 + ov)(2 diis_max + 1) + P + diis_max^2 doubles plus a 72-byte header;
 * thc_save_checkpoint writes it to host memory, thc_load_checkpoint restores it (THC_EINVAL for
 * a buffer that is not a checkpoint of a context with the same nP, o v and diis_max).  A resumed
 * FP64 solve repeats the uninterrupted one's iterations exactly; a mixed-precision one restarts
 * its precision ladder.  Host buffers; both calls synchronize the stream. */
int thc_checkpoint_bytes(thc_ctx* ctx, size_t* bytes);
int thc_save_checkpoint(thc_ctx* ctx, void* host, size_t bytes);
int thc_load_checkpoint(thc_ctx* ctx, const void* host, size_t bytes);

/* Per iteration of the last thc_iterate call, THC_ITER_* bits: the residual was mixed precision;
 * the iteration started from the MP2 guess after a divergence; DIIS dropped vectors to keep its
 * subspace well conditioned.  flags[max] host; *count receives the number of iterations. */
#define THC_ITER_MIXED 1
#define THC_ITER_RESTARTED 2
#define THC_ITER_DIIS_DROPPED 4
#define THC_ITER_LEARNED 8  /* the iteration descends from the learned start (thc_options.guess = 1) */
int thc_history_flags(const thc_ctx* ctx, int max, int* flags, int* count);

/* Per-iteration record of the last thc_iterate call (host arrays of length >= max, any may be
 * NULL): energy and residual norm of the amplitudes evaluated at each iteration and the wall
 * time in seconds from the start of the call to the end of that iteration's evaluation.
 * *count receives the number of iterations recorded (at most max are copied). */
int thc_history(const thc_ctx* ctx, int max, double* energy, double* rnorm, double* seconds, int* count);

/* Correlation energy of the current state (host scalar), the usual CCSD expression
 * sum (t_ij^ab + t_i^a t_j^b)(2(ia|jb) - (ib|ja)) with Cholesky integrals. */
int thc_energy(thc_ctx* ctx, double* e_corr);
/* Per iteration of the last thc_iterate call: 1 where the residual was evaluated in mixed
 * precision, 0 where in FP64.  mixed[max] host; *count receives the number of iterations. */
int thc_history_precision(const thc_ctx* ctx, int max, int* mixed, int* count);

/* Current state in the raw basis: Z [nP][nP], t1 [o][v] (device; either may be NULL). */
int thc_get_state(thc_ctx* ctx, double* Z, double* t1);
/* Replaces the state (t1 may be NULL = zero); clears the DIIS history. */
int thc_set_state(thc_ctx* ctx, const double* Z, const double* t1);

/* Device working memory held by the context (bytes), valid after thc_build_factors. */
int thc_memory_bytes(const thc_ctx* ctx, size_t* bytes);

/* How the context evaluates a residual, valid after thc_build_factors: the blocking of the
 * paper's loops (the fused pass over Cholesky vectors A of Alg. 1-3 and 8, the X-blocked and
 * grid-chunked Alg. 6, the X-chunked Alg. 7) and the kernel paths they take. */
typedef struct thc_plan_info {
  int64_t a_block;        /* Cholesky vectors per fused-pass block */
  int64_t alg1_splits;    /* K slices of the symmetric product sum_A C^A T C^A^T (Alg. 1) */
  int64_t alg1_tile;      /* tile edge of that product on the matrix cores (64 or 128) */
  int64_t x_block;        /* amplitude ranks X per H block (Alg. 6) */
  int64_t x_blocks;       /* H blocks per residual */
  int64_t i_chunk;        /* ERI grid points per H-kernel pass */
  int64_t i_chunks;       /* H-kernel passes per H block */
  int64_t h_generations;  /* H-kernel dispatches per pass (one per generation of resident tiles; odd
                             generations walk the grid points backwards) */
  int64_t h_tiles;        /* H-kernel tiles per pass (X tile x Y block x Z slice, Z >= Y) */
  int64_t x_chunk;        /* amplitude ranks X per batch of the two-GEMM exchange (Q x Q intermediates) */
  int64_t x7_chunk;       /* amplitude ranks X per chunk of the Alg. 7 intermediates */
  int64_t x7_chunks;      /* such chunks per residual */
  int32_t exchange_fused; /* 1: the fused Alg. 7 exchange kernel, 0: its two-GEMM form */
  int32_t lvv_resident;   /* 1: the vv Cholesky block is held in device memory */
  int32_t quintic;        /* 1: Eq. 32 + 33 by Alg. 4 and 5 (O(N^5)), 0: by Alg. 6 */
  int32_t reserved;
  int64_t q_pairs;        /* Alg. 4 and 5: pairs per batched product */
  int64_t q_jchunk;       /* Alg. 4 and 5: occupied j per chunk of the dense residual */
  uint64_t device_bytes;  /* device working memory */
} thc_plan_info;
int thc_plan(const thc_ctx* ctx, thc_plan_info* out);
/* The plan thc_build_factors would make for these options within budget_bytes of device memory
 * (synthetic != 0: inputs from thc_set_synthetic), without creating a context or touching device
 * memory; device_bytes is the working memory it needs (the workspace size for
 * thc_create_with_workspace).  The H-kernel generation count uses the current device, or the
 * MI355X's 64 resident tiles per XCD when there is none.  THC_ENOMEM if nothing fits. */
int thc_plan_query(const thc_options* opt, int synthetic, uint64_t budget_bytes, thc_plan_info* out);

/* Kernel timing with HIP events on the context stream.  thc_profile(ctx, 1) starts recording
 * (and clears earlier records); thc_profile_get synchronizes and returns, for the kernel
 * class `name` ("h_kernel", "gemm", "misc", or "residual" for whole residual evaluations),
 * the summed duration in milliseconds and the number of launches recorded. */
int thc_profile(thc_ctx* ctx, int enable);
int thc_profile_get(thc_ctx* ctx, const char* name, double* total_ms, int64_t* launches);
/* Flops (2 K per distinct output: 2 M N K per product, N (N + 1) K for a symmetric product whose
 * lower triangle is mirrored; counted once however the product is evaluated) issued to the MFMA
 * GEMM kernels since profiling was enabled, split into FP64, FP32 and split-BF16 products (any
 * pointer may be NULL). */
int thc_profile_flops(const thc_ctx* ctx, double* fp64_flops, double* fp32_flops, double* bf16x3_flops);

/* The library's FP64 MFMA GEMM (exposed for testing): C = alpha op(A) op(B) + beta C,
 * row-major, op = transpose when trans* != 0, batched with element strides sA, sB, sC (0: one
 * matrix shared by the batch).  Device arrays.  M, N or batch 0: nothing is done.  THC_EINVAL
 * for negative sizes or strides, a NULL operand, or a leading dimension shorter than its rows
 * (lda < K, or M when transA; ldb < N, or K when transB; ldc < N). */
int thc_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double* A,
              int64_t lda, int64_t sA, const double* B, int64_t ldb, int64_t sB, double beta, double* C,
              int64_t ldc, int64_t sC, int64_t batch, void* stream);

const char* thc_last_error(const thc_ctx* ctx);
void thc_destroy(thc_ctx* ctx);

/* ---- Learned starting guess -------------------------------------------------------------------
 * Not part of the paper: a small network proposes, per rank index P of the pseudo-canonical
 * working basis (E_mat w = e S w), a diagonal scaling c_P of the MP2 guess and a shift delta_P of
 * the Jacobi denominators.  The plain MP2 guess with delta = 0 stays the fallback.  All arrays
 * are device pointers unless stated otherwise. */
#define THC_GUESS_FEATURES 10

/* phi[nP][10] (FP32) from the current state T^ (after thc_build_factors: the MP2 guess):
 * [T^_PP, e_P, T^_PP e_P, eps_HOMO, eps_LUMO, mean eps_occ, mean eps_vir, nP / o,
 *  ||T^||_F / sqrt(nP), sum_Q |T^_PQ|]. */
int thc_guess_features(thc_ctx* ctx, float* phi);

/* pred[nP][ld] (FP32): column 0 is c_P, column 1 (if ld >= 2) is delta_P.  Sets
 * T^ <- diag(1 + c) T^ diag(1 + c) (and Z accordingly), and, if ld >= 2, the Jacobi denominators
 * D_PQ = max(e_P + e_Q + delta_P + delta_Q, (e_P + e_Q) / 2) for later thc_iterate calls.
 * Clears the DIIS history. */
int thc_guess_apply(thc_ctx* ctx, const float* pred, int64_t ld);

/* delta[nP] (FP64) as above, or NULL for the plain denominators e_P + e_Q.  Clears DIIS. */
int thc_set_shift(thc_ctx* ctx, const double* delta);

/* The current state in the working basis, T^[nP][nP], and (if sigma_hat is not NULL) the
 * projected residual of that state in the working basis, sigma^ = W^T sigma W.  Either may be NULL. */
int thc_working(thc_ctx* ctx, double* Th, double* sigma_hat);

/* Training targets of one converged system (all [nP][nP] in the working basis): Th0 the guess,
 * Tstar the converged state, sig0 the projected residual at the guess.  Writes c[nP], the
 * least-squares diagonal scaling of Th0 onto Tstar (Gauss-Newton), and delta[nP], the
 * least-squares secant fit -sig0 = (e_P + e_Q + delta_P + delta_Q)(Tstar - Th0).  Host FP64.
 * THC_ESINGULAR if a normal matrix is not positive definite. */
int thc_guess_targets(thc_ctx* ctx, const double* Th0, const double* Tstar, const double* sig0, double* c,
                      double* delta);

/* The network: n_in -> width -> width -> n_out, SiLU hidden activations, inputs standardized by
 * (x - mu_in) / sd_in and outputs produced as y_n sd_out + mu_out.  FP32 parameters in one flat
 * vector [W1 (n_in x width, row-major), b1, W2 (width x width), b2, W3 (width x n_out), b3],
 * Glorot-uniform initial weights from `seed`, zero biases.  Bound to `stream` (hipStream_t). */
typedef struct thc_mlp thc_mlp;

/* The network whose prediction starts the first thc_iterate after thc_build_factors when
 * thc_options.guess = 1 (features of the MP2 guess as thc_guess_features, BF16 inference as
 * thc_mlp_infer, applied as thc_guess_apply, all on the context's stream; a divergence or stall
 * from that start restarts from the MP2 guess with the plain denominators, see thc_iterate).  The network must have 10
 * inputs, width 256 and 1 or 2 outputs; it is not owned and must outlive its use.  NULL detaches
 * it.  thc_iterate returns THC_ESTATE if guess = 1 and no network is attached, THC_EINVAL if
 * nP^2 + o v < 6 nP (too small to stage the features). */
int thc_set_guess_network(thc_ctx* ctx, thc_mlp* net);
int thc_mlp_create(int64_t n_in, int64_t width, int64_t n_out, uint64_t seed, void* stream, thc_mlp** out);
/* Host arrays: mu_in, sd_in [n_in]; mu_out, sd_out [n_out]; scales must be positive. */
int thc_mlp_set_norm(thc_mlp* net, const float* mu_in, const float* sd_in, const float* mu_out, const float* sd_out);
/* Standardization fitted to training data X[rows][n_in], T[rows][n_out] (device): per-column
 * mean and standard deviation; a column with no spread gets sd = 1. */
int thc_mlp_fit_norm(thc_mlp* net, const float* X, const float* T, int64_t rows);
/* The standardization in use, copied to host arrays [n_in], [n_in], [n_out], [n_out]. */
int thc_mlp_get_norm(thc_mlp* net, float* mu_in, float* sd_in, float* mu_out, float* sd_out);
int thc_mlp_num_params(const thc_mlp* net, int64_t* n);
int thc_mlp_get_params(thc_mlp* net, float* p);       /* p[n] device */
int thc_mlp_set_params(thc_mlp* net, const float* p); /* p[n] device; resets the Adam moments */
/* FP32 forward: X[rows][n_in] -> Y[rows][n_out]. */
int thc_mlp_forward(thc_mlp* net, const float* X, int64_t rows, float* Y);
/* loss = mean over rows and outputs of (y_n - (T - mu_out) / sd_out)^2 (host float, may be NULL)
 * and its gradient grad[n] (device, may be NULL), FP32. */
int thc_mlp_loss_grad(thc_mlp* net, const float* X, const float* T, int64_t rows, float* loss, float* grad);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the loss above. */
int thc_mlp_train_step(thc_mlp* net, const float* X, const float* T, int64_t rows, float lr, float* loss);
/* The FP32 forward pass above without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops): the same kernels and result as
 * thc_mlp_forward, with the activations in a fixed device array of THC_MLP_SCRATCH_BYTES per GPU
 * (held until the process ends) instead of buffers the network allocates.  Row limit: about
 * THC_MLP_SCRATCH_BYTES / (4 (n_in + 2 width + n_out)), less the padding that starts each of the
 * four activation buffers on a 256-byte boundary (16 008 rows for 10 -> 256 -> 2); more rows
 * return THC_EINVAL with the limit in thc_mlp_last_error and launch nothing.  The array
 * is shared by every call on a GPU and keeps the last call's contents (nothing in it has to start
 * at zero): calls that overlap on one GPU (two streams or two threads) race. */
#define THC_MLP_SCRATCH_BYTES (32u << 20)
int thc_mlp_forward_noalloc(thc_mlp* net, const float* X, int64_t rows, float* Y);
/* BF16 inference on MFMA with FP32 accumulation (width 256, n_in <= 16, n_out <= 16). */
int thc_mlp_infer(thc_mlp* net, const float* X, int64_t rows, float* Y);
const char* thc_mlp_last_error(const thc_mlp* net);
void thc_mlp_destroy(thc_mlp* net);

#ifdef __cplusplus
}
#endif
#endif /* THC_H */
