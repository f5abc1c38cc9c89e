/*
 * amoeba.h — C ABI of the MI355X induced-dipole solver.
 *
 * The library solves for the induced dipoles mu of a Thole-damped point-dipole
 * polarizable force field (AMOEBA type) in a periodic orthorhombic box,
 *
 *     (alpha^-1 - T) mu = E_perm,
 *
 * by preconditioned conjugate gradient with the diagonal preconditioner
 * (paper: "Optimizations opportunities", the PCG of the polarization solver,
 * and "Performance and Scalability Results" for the diagonal preconditioner
 * and the convergence threshold).  T mu is the full Ewald field of the
 * dipoles: a real-space, Thole-damped, erfc-screened pair sum within a sharp
 * cutoff over a blocked neighbour list (paper: "Neighbor list", "Box
 * partitioning", "List filtering"), a smooth-PME reciprocal part (paper:
 * "Reciprocal space scheme": B-spline spread, forward FFT, scalar product,
 * backward FFT, gather), and the Gaussian self field 4 beta^3/(3 sqrt(pi)) mu.
 * Mixed precision (paper: "Precision study and Validation") computes pair and
 * PME arithmetic in FP32 and accumulates fields in 64-bit fixed point, while
 * the PCG vectors, dot products and convergence test stay FP64.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (HIP device memory, e.g. from a torch
 *    tensor), contiguous, row-major, in the caller's atom order; the library
 *    permutes internally and never keeps or frees caller memory.  Scalar
 *    outputs (energy, iteration count) are HOST pointers.
 *  - Per-atom vectors are FP64 N x 3 (x,y,z); quadrupoles FP64 N x 6 as the
 *    traceless Theta (point potential Theta:rr / r^5), order xx,xy,xz,yy,yz,zz.
 *  - Units: Angstrom, e, e*A, e*A^2, A^3; fields in e/A^2; energies in
 *    kcal/mol (C = 332.0637133 kcal*A/(mol e^2)); Debye only in tolerances
 *    (1 e*A = 4.80320 D).
 *  - All work is enqueued on the HIP stream given to amoeba_create; every call
 *    returns after its outputs are complete.  A context is not thread-safe: use
 *    one context per host thread.
 *  - Errors: every call returns an amoeba_status; negative values are errors
 *    with a message in amoeba_last_error().  Host-side argument checks run
 *    before any work is queued; checks that need the data (NaN/Inf, traceless
 *    quadrupoles, list staleness, field range) run on the device and are
 *    reported when the call returns.  On an error the outputs are unspecified.
 */
#ifndef AMOEBA_H
#define AMOEBA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct amoeba_ctx amoeba_ctx;

typedef enum amoeba_status {
    AMOEBA_OK = 0,
    AMOEBA_NOT_CONVERGED = 1,  /* outputs valid: mu is the last iterate, iterations = max_iter */
    AMOEBA_E_INVALID = -1,     /* bad argument or parameter (message says which)               */
    AMOEBA_E_NOMEM = -2,       /* device allocation failed or max_workspace_bytes exceeded      */
    AMOEBA_E_DEVICE = -3,      /* no usable gfx950 device, or a HIP / rocFFT call failed        */
    AMOEBA_E_LIST = -4,        /* block list missing or stale (an atom moved > buffer/2)        */
    AMOEBA_E_OVERFLOW = -5,    /* a field beyond the exact fixed-point range (|E| >= 8192 e/A^2) */
    AMOEBA_E_NUMERIC = -6,     /* NaN/Inf in an input, or a PCG breakdown                       */
    AMOEBA_E_STATE = -7        /* call order violated (e.g. no amoeba_set_atoms yet)             */
} amoeba_status;

typedef enum amoeba_precision {
    AMOEBA_FP64 = 0,   /* all arithmetic in FP64, FP64 atomics                                 */
    AMOEBA_MIXED = 1   /* FP32 pair/PME math, 64-bit fixed-point fields, FP64 PCG               */
} amoeba_precision;

typedef enum amoeba_guess_mode {
    AMOEBA_GUESS_ZERO = 0,     /* mu0 = 0                                                      */
    AMOEBA_GUESS_GIVEN = 1,    /* mu0 = mu_guess (e.g. the previous configuration's dipoles)   */
    AMOEBA_GUESS_LEARNED = 2,  /* mu0 from the learned per-atom network (amoeba_guess_*)       */
    AMOEBA_GUESS_BEST = 3      /* learned and given guesses both evaluated; the one with the
                                  smaller preconditioned initial residual is used (zero if
                                  mu_guess is NULL)                                           */
} amoeba_guess_mode;

/* How the reciprocal field is computed (paper, "Reciprocal space scheme"), for the induced
 * dipoles of the PCG product and for the permanent multipoles.  Both give the same field up to
 * rounding. */
typedef enum amoeba_pme_path {
    AMOEBA_PME_AUTO = 0,    /* planes when the grid fits, else bricks                          */
    AMOEBA_PME_PLANES = 1,  /* x-planes held in LDS: spread and y-z FFT fused, x-line FFT with
                               the influence function, inverse y-z FFT and interpolation fused;
                               needs every K a product of 2, 3, 5, 7 and a plane of
                               ceil(K1/2) x 2(K2/2+1) complex FP64 values within 150 KB       */
    AMOEBA_PME_BRICKS = 2   /* 8^3-point brick spread and gather around rocFFT r2c / c2r      */
} amoeba_pme_path;

/* How the real-space dipole product gets the radial coefficients B1', B2' of its in-cutoff
 * pairs (paper, PCG section: the option of computing and storing the real-space matrix elements
 * once before iterating).  The coefficients with the pair displacement give the interaction
 * tensor, -B1' I + B2' r r^T.  Both use bitwise the same coefficients, so that mixed-precision
 * products (exact fixed-point sums) are bitwise equal; FP64 products agree to the rounding of
 * their FP64 sums. */
typedef enum amoeba_pair_store {
    AMOEBA_PAIRS_AUTO = 0,     /* STORED in FP64, where the pair functions cost more than reading
                                  the coefficients back; COMPUTE in mixed precision, where the
                                  FP32 tiles are bound by LDS traffic that the store leaves as
                                  it is                                                         */
    AMOEBA_PAIRS_COMPUTE = 1,  /* every product evaluates erfc, the Thole damping and the powers
                                  of 1/r for every pair                                          */
    AMOEBA_PAIRS_STORED = 2    /* the first product after a new configuration (or new atom
                                  parameters) stores B1', B2' per pair (8 bytes per pair mixed, 16
                                  FP64); later products read them back and rebuild only the
                                  displacement.  Falls back to COMPUTE, per tile, where the store
                                  does not fit the workspace cap                                */
} amoeba_pair_store;

typedef struct amoeba_params {
    int32_t n_atoms;       /* N >= 1                                                          */
    double box[3];         /* orthorhombic box edges (A)                                      */
    double cutoff;         /* real-space cutoff rc (A); pairs with |r| < rc                   */
    double buffer;         /* neighbour-list buffer (A) >= 0; list is valid while every atom
                              stays within buffer/2 of its position at the last build        */
    double ewald_alpha;    /* Ewald splitting beta (1/A) > 0                                  */
    int32_t grid[3];       /* PME grid points per edge, 2*order <= K <= 2048 (FFT sizes of      
                              2, 3, 5, 7 factors are the fast ones)                           */
    int32_t order;         /* B-spline order; must be 5                                      */
    int32_t precision;     /* amoeba_precision                                                */
    int64_t max_workspace_bytes; /* cap on device memory the context may allocate; 0 = none  */
} amoeba_params;

typedef struct amoeba_info {
    int32_t n_atoms;
    int32_t n_blocks;          /* 64-atom blocks (last one padded with phantom atoms)           */
    int32_t n_tiles;           /* block x 64-atom tiles in the list (diagonal tiles included)  */
    int32_t precision;
    int64_t n_pairs;           /* in-cutoff unordered pairs at the last configuration           */
    int64_t workspace_bytes;   /* device memory held by the context                             */
    int32_t last_iterations;   /* PCG iterations of the last amoeba_polarize                    */
    double last_rms_debye;     /* final preconditioned-residual rms of the last solve (D)      */
    int32_t last_guess;        /* starting point the last solve used: an amoeba_guess_mode
                                  (ZERO, GIVEN or LEARNED; BEST resolves to one of them)        */
    int32_t guess_loaded;      /* 1 once amoeba_guess_set_model has been called                 */
    double last_guess_rms_debye[2]; /* AMOEBA_GUESS_BEST: rms of alpha r0 (D) of the fallback
                                  (zero or given) [0] and of the learned guess [1]; else 0    */
    int32_t pair_min_image;    /* 1 if the pair kernels apply the minimum image per pair; 0 when
                                  the list build proved block-relative offsets already give it
                                  (cutoff + 3 buffer + 4 x largest block half-extent < box/2) */
    int32_t pme_planes;        /* 1 if the PCG products use the plane path (amoeba_pme_path)  */
    int32_t pair_store;        /* 1 if the dipole products replay stored pair coefficients
                                  (amoeba_pair_store)                                           */
    int64_t pair_store_bytes;  /* device memory held by the stored coefficients                 */
} amoeba_info;

/* Create a context for one system size and one parameter set on the current HIP device,
 * enqueueing on `hip_stream` (a hipStream_t; NULL = the default stream).  Validates the
 * parameters on the host first (AMOEBA_E_INVALID, no device touched), then checks the device
 * (AMOEBA_E_DEVICE unless it is gfx950), allocates the workspace and builds the PME tables and
 * FFT plans.  *out is set only on success. */
int amoeba_create(const amoeba_params* params, void* hip_stream, amoeba_ctx** out);

/* Release every device buffer and plan of the context.  NULL is accepted. */
int amoeba_destroy(amoeba_ctx* ctx);

/* Message of the last error on this context ("" if none); valid until the next call. */
const char* amoeba_last_error(const amoeba_ctx* ctx);

/* Message of the last amoeba_create failure in this thread (no context exists then). */
const char* amoeba_create_error(void);

/* Per-atom polarization parameters and the scaled pairs of the permanent field.
 *   alpha[N]  polarizabilities (A^3) > 0;  thole[N] Thole a >= 0 (pair uses min(a_i, a_j)).
 *   sc_ptr[N+1], sc_j[n_scaled], sc_s[n_scaled]: CSR of pairs whose permanent-field interaction
 *   is multiplied by s (s = 0 excludes the pair; AMOEBA's polarization p-scale).  Both
 *   directions of every pair must be listed with the same s; j != i.  The correction is applied
 *   at any separation (paper, final real-space scheme: scaled interactions are corrected in a
 *   separate pass).  The mutual dipole field T is never scaled (every pair Thole-damped).
 * Validated on the device (AMOEBA_E_INVALID names the first violation). */
int amoeba_set_atoms(amoeba_ctx* ctx, const double* alpha, const double* thole,
                     const int32_t* sc_ptr, const int32_t* sc_j, const double* sc_s,
                     int64_t n_scaled);

/* Build the blocked neighbour list for positions pos[N][3] (paper "Box partitioning",
 * "List filtering"): atoms are sorted along a column-serpentine cell order into 64-atom blocks,
 * block pairs within cutoff + buffer are found, and for every block the atoms of later blocks
 * within cutoff + buffer of any of its atoms are packed into 64-atom tiles.  Positions may lie
 * outside the box (they are wrapped). */
int amoeba_build_blocklist(amoeba_ctx* ctx, const double* pos);

/* Keep the blocked neighbour list valid for positions pos[N][3] (paper "Neighbor list": the
 * list holds the pairs within cutoff + buffer so that it need not be rebuilt at every time
 * step).  The list is rebuilt (as amoeba_build_blocklist) only when none exists or when an atom
 * has moved more than buffer/2 from where it was at the last build; otherwise only the
 * per-configuration in-cutoff masks are refreshed for pos.  *rebuilt_out (may be NULL) is set
 * to 1 when the list was rebuilt, else 0.  Errors as amoeba_build_blocklist. */
int amoeba_update_blocklist(amoeba_ctx* ctx, const double* pos, int32_t* rebuilt_out);

/* Permanent field E_perm[N][3] (e/A^2) of charges q[N], dipoles dip[N][3] and traceless
 * quadrupoles quad[N][6] at positions pos (paper "Global scheme": real space + reciprocal
 * space): real-space tiles with Thole damping lambda3/5/7, the scaled-pair correction at any
 * separation, smooth PME of the multipolar density, and the dipole self field. */
int amoeba_perm_field(amoeba_ctx* ctx, const double* pos, const double* q, const double* dip,
                      const double* quad, double* e_perm);

/* out[N][3] = (alpha^-1 - T) mu for dipoles mu[N][3] (e*A) at positions pos: one matrix-vector
 * product of the PCG (paper "Optimizations opportunities": the polarization matrix-vector
 * product of every iteration). */
int amoeba_dipole_matvec(amoeba_ctx* ctx, const double* pos, const double* mu, double* out);

/* The two parts of T mu separately: e_real[N][3] the real-space pair field and e_recip[N][3]
 * the smooth-PME reciprocal field (without the self term).  Either pointer may be NULL.
 * Diagnostic entry: the same kernels as amoeba_dipole_matvec. */
int amoeba_dipole_field_parts(amoeba_ctx* ctx, const double* pos, const double* mu,
                              double* e_real, double* e_recip);

/* Solve (alpha^-1 - T) mu = e_perm by PCG with z = alpha r, stopping when the rms over atoms
 * of z is below tol_debye (Debye), or after max_iter iterations (AMOEBA_NOT_CONVERGED; mu_out
 * is then the last iterate).  guess_mode selects mu0 (mu_guess may be NULL for ZERO/LEARNED).
 * Outputs: mu_out[N][3] (device, e*A); *e_pol_out = -1/2 C sum_i mu_i . e_perm_i (host,
 * kcal/mol); *iters_out = matrix-vector products after the initial residual (host).  In mixed
 * precision the true residual e_perm - A mu is recomputed once the recursive one passes the
 * tolerance (iteration continues if it does not), unless the recursion cannot have drifted by
 * a tenth of the tolerance (amoeba_set_residual_check). */
int amoeba_polarize(amoeba_ctx* ctx, const double* pos, const double* e_perm,
                    const double* mu_guess, int32_t guess_mode, double tol_debye, int32_t max_iter,
                    double* mu_out, double* e_pol_out, int32_t* iters_out);

/* One configuration of a trajectory in one call (paper "Global scheme": the permanent field,
 * then the induced dipoles, at every step; "Neighbor list": the list kept while the buffer
 * allows): amoeba_update_blocklist(pos), amoeba_perm_field(pos, q, dip, quad) and
 * amoeba_polarize(pos, E_perm, mu_guess, guess_mode, ...) with the same meaning of every
 * argument and output, with E_perm handed to the solve in the library's own atom order and
 * without the host waits between the three.  e_perm_out[N][3] (may be NULL) receives E_perm;
 * *rebuilt_out (may be NULL) is 1 when the list was rebuilt.  The DELTA kind of the learned
 * start uses the reference set by amoeba_guess_set_reference.  Errors of the permanent field
 * (a quadrupole not traceless, a non-finite multipole, the fixed-point range) are reported in
 * preference to the solve's; on any error the outputs are unspecified. */
int amoeba_polarize_configuration(amoeba_ctx* ctx, const double* pos, const double* q, const double* dip,
                                  const double* quad, const double* mu_guess, int32_t guess_mode,
                                  double tol_debye, int32_t max_iter, double* e_perm_out, double* mu_out,
                                  double* e_pol_out, int32_t* iters_out, int32_t* rebuilt_out);

/* ------------------------------------------------------------------------------------------
 * Two induced-dipole sets (AMOEBA's full polarization model; paper "Real space scheme": every
 * AMOEBA polarization interaction carries three scaling factors).  mu_d answers the permanent
 * field with the direct scales d, mu_p the field with the polarization scales p (the scales of
 * amoeba_set_atoms); the mutual operator (alpha^-1 - T) is the same for both (u-scale 1:
 * every pair Thole-damped, unscaled), and E_pol = -1/2 C mu_d . e_p (= -1/2 C mu_p . e_d, the
 * operator being symmetric).
 * ------------------------------------------------------------------------------------------ */

/* Direct scales sc_s_d[n_scaled] of the pairs listed by amoeba_set_atoms, in the same CSR order
 * (device FP64); n_scaled must equal the count given there.  Validated like the p-scales
 * (finite, both directions of a pair equal).  Without this call (or after a new
 * amoeba_set_atoms, which drops them) the direct scales equal the p-scales. */
int amoeba_set_direct_scales(amoeba_ctx* ctx, const double* sc_s_d, int64_t n_scaled);

/* The two permanent fields e_d[N][3] (direct scales) and e_p[N][3] (p-scales) of one set of
 * multipoles, as amoeba_perm_field computes e_perm (which equals e_p): the unscaled real-space
 * tiles, the reciprocal part and the self field are shared, the scaled-pair corrections differ.
 * Errors as for amoeba_perm_field. */
int amoeba_perm_field_dp(amoeba_ctx* ctx, const double* pos, const double* q, const double* dip,
                         const double* quad, double* e_d, double* e_p);

/* Both sets: (alpha^-1 - T) mu_d = e_d and (alpha^-1 - T) mu_p = e_p, each by the PCG of
 * amoeba_polarize from zero to tol_debye (the same stopping rule; in mixed precision with its
 * true-residual check).  Outputs: mu_d_out, mu_p_out [N][3] (device, e*A); *e_pol_out =
 * -1/2 C sum_i mu_d,i . e_p,i (host, kcal/mol; may be NULL); iters_out[2] (host; may be NULL):
 * the iterations of the d and the p solve.  AMOEBA_NOT_CONVERGED if either stopped at max_iter
 * (both outputs are then the last iterates).  Errors as for amoeba_polarize. */
int amoeba_polarize_dp(amoeba_ctx* ctx, const double* pos, const double* e_d, const double* e_p,
                       double tol_debye, int32_t max_iter, double* mu_d_out, double* mu_p_out,
                       double* e_pol_out, int32_t* iters_out);

/* Gradient of the polarization energy with respect to the positions, grad_out[N][3] =
 * dE_pol/dr (device FP64, kcal/mol/A; the polarization forces are its negative), for the
 * permanent multipoles (q, dip, quad, as for amoeba_perm_field) and the induced dipoles mu[N][3]
 * (device, e*A) at positions pos (paper "Global scheme": the polarization solve and its forces
 * make the non-bonded step; "Real space scheme": scaled pairs corrected separately).  The result
 * is the gradient of E_pol = -1/2 C mu.E_perm at dipoles that solve the system, where E_pol is
 * stationary in mu:
 *     dE_pol/dr_k = C [ -1/2 mu.(dT/dr_k) mu - mu.(dE_perm/dr_k) ],
 * with the real-space pairs (Thole damping up to lambda9 for the quadrupole terms, the p-scale of
 * the listed pairs in the permanent terms, unscaled mutual terms) and the smooth-PME terms
 * (second and third B-spline derivatives on the grid potentials of the dipoles and of the
 * multipoles).  For dipoles that do not solve the system it is the partial derivative at fixed
 * mu.  Mixed precision: FP32 pair and PME arithmetic (near-coincident pairs below 0.5 A in FP64),
 * fixed-point pair sums; the grid uses the brick spread and rocFFT in either precision.
 * Errors as for amoeba_perm_field (traceless check, non-finite inputs, the fixed-point range). */
int amoeba_polarization_gradient(amoeba_ctx* ctx, const double* pos, const double* q, const double* dip,
                                 const double* quad, const double* mu, double* grad_out);

/* ------------------------------------------------------------------------------------------
 * Learned initial guess (an addition to the paper's method: the paper starts PCG from a plain
 * guess).  A small per-atom network over neighbour-list environment features predicts the
 * induced dipoles; amoeba_polarize can start from its prediction (AMOEBA_GUESS_LEARNED) or from
 * whichever of the prediction and the zero / given guess has the smaller preconditioned
 * initial residual (AMOEBA_GUESS_BEST).  PCG always converges to the same tolerance, so the
 * guess changes the iteration count, never the accepted accuracy.
 *
 * Bases (e*A, per atom), with R the real-space Thole-damped Ewald dipole field over the
 * in-cutoff pairs (the real-space part of T) and c = 4 beta^3 / (3 sqrt(pi)):
 *     v0 = alpha E_perm,  v1 = alpha (R[v0] + c v0),  v2 = alpha (R[v1] + c v1)
 * (the first terms of the Neumann series of (alpha^-1 - T)^-1 E_perm without the reciprocal
 * part).  Invariant features x[AMOEBA_GUESS_NFEAT]:
 *     alpha, Thole a, D|v0|, D|v1|, D|v2| (D = 4.80320 Debye per e*A),
 *     cos(v0,v1), cos(v0,v2), cos(v1,v2) with cos(a,b) = a.b / sqrt(|a|^2 |b|^2 + 1e-20),
 *     sum over in-cutoff neighbours of exp(-((r - c_k) / 0.6 A)^2) for c_k = 1, 2, 3 A.
 * Network (FP32): xh = (x - mean) * inv_std; h1 = silu(W1 xh + b1); h2 = silu(W2 h1 + b2);
 * y = W3 h2 + b3; mu0 = sum_k (s_k + y_k) v_k, s = (1, 1, 1) for these bases (the DELTA kind
 * below has its own bases and offsets).  Loss of a batch of n samples:
 * L = D^2 / n * sum_i |mu0_i - target_i|^2 (Debye^2).  Optimiser: Adam (beta1 0.9, beta2 0.999,
 * eps 1e-8, bias-corrected).
 *
 * Model vector (FP32, AMOEBA_GUESS_NMODEL floats, row-major): W1[64][11], b1[64], W2[64][64],
 * b2[64], W3[3][64], b3[3], mean[11], inv_std[11].  The first AMOEBA_GUESS_NPARAM entries are
 * trained; the last 2*NFEAT are set by amoeba_guess_fit_norm.
 *
 * Training-set arrays are caller-owned device memory in sample order: feat[n][NFEAT] FP32,
 * basis[n][NBASIS][3] FP32 (e*A), target[n][3] FP32 (e*A).  Batches are either the first n_batch
 * rows (idx NULL) or the rows idx[0..n_batch) (int32 device array; every entry must lie in
 * [0, n_rows), else AMOEBA_E_INVALID).  Sums over samples run in a fixed order, so every call
 * is bitwise reproducible.
 * ---------------------------------------------------------------------------------------- */
#define AMOEBA_GUESS_NFEAT 11
#define AMOEBA_GUESS_NBASIS 3
#define AMOEBA_GUESS_HIDDEN 64
#define AMOEBA_GUESS_NPARAM 5123   /* 64*11 + 64 + 64*64 + 64 + 3*64 + 3 */
#define AMOEBA_GUESS_NMODEL 5145   /* NPARAM + 2*NFEAT                   */

/* Which bases the network combines (the kind is a setting of the context, kept across
 * amoeba_guess_set_model; the default is NEUMANN):
 *   AMOEBA_GUESS_KIND_NEUMANN  the bases above, offsets s = (1, 1, 1); needs only the
 *                              configuration (two real-space products per guess).
 *   AMOEBA_GUESS_KIND_DELTA    for a configuration that follows a solved one, whose converged
 *                              dipoles mu_ref and permanent field E_ref are given by
 *                              amoeba_guess_set_reference: v0 = mu_ref, v1 = alpha (E_perm -
 *                              E_ref), v2 = alpha E_perm, offsets s = (1, 0, 0), so that the
 *                              untrained network returns mu_ref (the previous-step guess); no
 *                              real-space product.  The three radial features are zero (left
 *                              out: the walk over the tiles costs more than the guess saves).
 * mu0 = sum_k (s_k + y_k) v_k in both; the other features are the same functions of the bases. */
typedef enum amoeba_guess_kind {
    AMOEBA_GUESS_KIND_NEUMANN = 0,
    AMOEBA_GUESS_KIND_DELTA = 1
} amoeba_guess_kind;

/* Select the kind for later features, predictions, training steps and learned starts.
 * Unknown kind: AMOEBA_E_INVALID. */
int amoeba_guess_set_kind(amoeba_ctx* ctx, int32_t kind);

/* Reference configuration of the DELTA kind: mu_ref[N][3] (e*A) and e_ref[N][3] (e/A^2),
 * device FP64 in caller atom order, copied into the context on its stream (the caller may
 * reuse its arrays once the stream has passed the copy; no host wait).  Needed before any
 * DELTA feature, prediction or learned start (else AMOEBA_E_STATE); a non-finite entry makes
 * the call that uses it return AMOEBA_E_NUMERIC. */
int amoeba_guess_set_reference(amoeba_ctx* ctx, const double* mu_ref, const double* e_ref);

/* Load a model (host array of n_floats == AMOEBA_GUESS_NMODEL floats); resets the Adam
 * moments and step count.  The first call allocates the guess workspace. */
int amoeba_guess_set_model(amoeba_ctx* ctx, const float* model, int64_t n_floats);

/* Copy the current model to a host array of n_floats == AMOEBA_GUESS_NMODEL floats. */
int amoeba_guess_get_model(amoeba_ctx* ctx, float* model, int64_t n_floats);

/* Checkpoint of the learned guess: a versioned host blob holding the kind, the model, the
 * Adam moments and the Adam step count, so that training resumes exactly where it stopped.
 * Layout (little-endian): char magic[8] = "AMGUESS" (NUL-terminated); uint32 version
 * (AMOEBA_GUESS_BLOB_VERSION); int32 kind; int32 NFEAT, NBASIS, HIDDEN, NPARAM, NMODEL;
 * int32 0; int64 Adam step count; float model[NMODEL]; float adam_m[NPARAM];
 * float adam_v[NPARAM]  (AMOEBA_GUESS_BLOB_BYTES bytes in all).
 * amoeba_guess_save: blob NULL -> *bytes = the size needed; else *bytes must be at least
 * that size (AMOEBA_E_INVALID otherwise) and receives the size written.  Needs a loaded model.
 * amoeba_guess_load: a blob of another version, kind, shape or size, or with non-finite
 * entries, is rejected (AMOEBA_E_INVALID / AMOEBA_E_NUMERIC) and leaves the context as it was. */
#define AMOEBA_GUESS_BLOB_VERSION 1
#define AMOEBA_GUESS_BLOB_BYTES (48 + 4 * (AMOEBA_GUESS_NMODEL + 2 * AMOEBA_GUESS_NPARAM))
int amoeba_guess_save(amoeba_ctx* ctx, void* blob, int64_t* bytes);
int amoeba_guess_load(amoeba_ctx* ctx, const void* blob, int64_t bytes);

/* Bases and features of one configuration (positions pos, permanent field e_perm, the list
 * built; the reference set for the DELTA kind): feat_out[N][NFEAT] and basis_out[N][NBASIS][3]
 * (device FP32, caller atom order). */
int amoeba_guess_features(amoeba_ctx* ctx, const double* pos, const double* e_perm,
                          float* feat_out, float* basis_out);

/* Set the model's mean and inv_std from the first n_rows rows of feat (population standard
 * deviation; inv_std = 0 where it is <= 1e-6).  Needs a loaded model. */
int amoeba_guess_fit_norm(amoeba_ctx* ctx, const float* feat, int64_t n_rows);

/* mu_out[n][3] (device FP32, e*A) = the network's prediction for the n rows of feat/basis. */
int amoeba_guess_forward(amoeba_ctx* ctx, const float* feat, const float* basis, int64_t n,
                         float* mu_out);

/* Loss and gradient of a batch without changing the model: grad_out[NPARAM] (device FP32),
 * *loss_out (host, Debye^2). */
int amoeba_guess_gradient(amoeba_ctx* ctx, const float* feat, const float* basis,
                          const float* target, int64_t n_rows, const int32_t* idx, int64_t n_batch,
                          float* grad_out, double* loss_out);

/* amoeba_guess_gradient for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same kernels and the same
 * result, bitwise, but the per-workgroup partials, the loss and the flag word live in a
 * library-owned static device array of about 2.5 MiB per GPU (held from the first
 * amoeba_create on that GPU until the process ends) instead of context memory; no allocation,
 * no memset node.  n_batch at most AMOEBA_GUESS_NOALLOC_MAX_BATCH, else AMOEBA_E_INVALID.
 * Every call on a GPU shares that GPU's array: calls that overlap on one GPU (several host
 * threads, several streams) race, so the caller serialises them.  Needs a loaded model. */
#define AMOEBA_GUESS_NOALLOC_MAX_BATCH 8192
int amoeba_guess_gradient_noalloc(amoeba_ctx* ctx, const float* feat, const float* basis,
                                  const float* target, int64_t n_rows, const int32_t* idx,
                                  int64_t n_batch, float* grad_out, double* loss_out);

/* One Adam step with learning rate lr on a batch; *loss_out (host, may be NULL) is the batch
 * loss before the step. */
int amoeba_guess_train_step(amoeba_ctx* ctx, const float* feat, const float* basis,
                            const float* target, int64_t n_rows, const int32_t* idx,
                            int64_t n_batch, float lr, double* loss_out);

/* The learned guess for one configuration: mu0_out[N][3] (device FP64, caller order), the
 * starting point amoeba_polarize uses with AMOEBA_GUESS_LEARNED. */
int amoeba_guess_predict(amoeba_ctx* ctx, const double* pos, const double* e_perm, double* mu0_out);

/* Select the reciprocal dipole-field path (amoeba_pme_path) for later products.
 * AMOEBA_PME_PLANES on a grid that does not fit: AMOEBA_E_INVALID, the setting is unchanged.
 * The default is AMOEBA_PME_AUTO. */
int amoeba_set_pme_path(amoeba_ctx* ctx, int32_t path);

/* Run each PCG iteration (the dipole product on its two streams, the update and the direction
 * kernels) as one captured HIP graph (enable != 0) or as individual launches (enable = 0, the
 * default).  The paper observes that the small kernels of an iteration are launch bound; a graph
 * replays them without per-kernel host launches.  Both give bitwise the same iterates: the graph
 * holds the same kernels with the same arguments.  On MI355X the graph measured slower than the
 * direct launches, which the host already queues two iterations ahead (water_96000 solve 1.49
 * against 1.45 ms), hence the default.  The graph is used on the plane PME path without stage
 * timers; it is captured at the first iteration that can use it and captured again when a
 * launch parameter it holds changes (pair kernel variant, coefficient store).  Waits for the
 * context stream.  A capture that fails turns graphs off for the context (the solve goes on with
 * direct launches). */
int amoeba_set_graphs(amoeba_ctx* ctx, int32_t enable);

/* When a mixed-precision solve recomputes its true residual after the recursive one has passed
 * the tolerance.  The recursion drifts from e - A mu by the rounding of the products; with their
 * relative error below eps = 1e-5 (above three times the bar the products are tested to against
 * the FP64 oracle) the drift in z = alpha r is at most 2 eps sum_k rms(z_k) over the iterates.
 *   AMOEBA_RESIDUAL_CHECK_AUTO    (default) recompute only when that bound exceeds a tenth of
 *                                 the tolerance (a start far from the solution, e.g. zero)
 *   AMOEBA_RESIDUAL_CHECK_ALWAYS  recompute after every mixed-precision solve
 * A check that passes leaves the outputs as they were.  Unknown mode: AMOEBA_E_INVALID. */
typedef enum amoeba_residual_check {
    AMOEBA_RESIDUAL_CHECK_AUTO = 0,
    AMOEBA_RESIDUAL_CHECK_ALWAYS = 1
} amoeba_residual_check;
int amoeba_set_residual_check(amoeba_ctx* ctx, int32_t mode);

/* Select how the real-space dipole product gets its pair coefficients (amoeba_pair_store) for
 * later products; an unknown value: AMOEBA_E_INVALID.  The default is AMOEBA_PAIRS_AUTO. */
int amoeba_set_pair_store(amoeba_ctx* ctx, int32_t mode);

/* Sizes and counters of the context (host struct). */
int amoeba_get_info(const amoeba_ctx* ctx, amoeba_info* out);

/* Kernel-time accounting (diagnostic; used by the benchmark for its roofline figures).
 * When enabled, every launch of the listed stages is bracketed by HIP events on the stream it
 * runs on; amoeba_get_timing synchronises the context stream and returns the accumulated
 * milliseconds and launch counts per stage since the last amoeba_set_timing.  Launches that
 * return early because the solve already converged are included (as a profiler would count
 * them); `matvecs` counts the matrix-vector products that did work. */
typedef enum amoeba_stage {
    AMOEBA_T_LIST = 0,     /* list build and per-configuration mask refresh                 */
    AMOEBA_T_PERM = 1,     /* permanent-field tiles and assembly                            */
    AMOEBA_T_REAL = 2,     /* real-space dipole tiles (one per matrix-vector product)       */
    AMOEBA_T_SPREAD = 3,   /* PME spread                                                    */
    AMOEBA_T_FFT = 4,      /* forward FFT + influence product + backward FFT                */
    AMOEBA_T_GATHER = 5,   /* PME gather fused with the operator assembly and p.Ap          */
    AMOEBA_T_PCG = 6,      /* PCG vector updates and reductions                             */
    AMOEBA_T_GUESS = 7,    /* learned guess: features, network, training kernels (the
                              real-space products of its bases count under AMOEBA_T_REAL)     */
    AMOEBA_T_COUNT = 8
} amoeba_stage;

typedef struct amoeba_timing {
    double ms[AMOEBA_T_COUNT];
    int64_t launches[AMOEBA_T_COUNT];
    int64_t matvecs;
} amoeba_timing;

/* enable: AMOEBA_TIMING_OFF, AMOEBA_TIMING_STAGES (every stage alone: the products run
 * their real-space and reciprocal parts one after the other on the context stream, so that
 * each stage's time is its own) or AMOEBA_TIMING_LIVE (only AMOEBA_T_REAL, on the second
 * stream where it runs beside the reciprocal passes; the products keep their overlap, and the
 * time includes the sharing of the GPU: two events per product, light enough to leave on in a
 * timed run).  Every call resets the counters; any other value: AMOEBA_E_INVALID. */
typedef enum amoeba_timing_mode {
    AMOEBA_TIMING_OFF = 0,
    AMOEBA_TIMING_STAGES = 1,
    AMOEBA_TIMING_LIVE = 2
} amoeba_timing_mode;
int amoeba_set_timing(amoeba_ctx* ctx, int enable);
int amoeba_get_timing(amoeba_ctx* ctx, amoeba_timing* out);

#ifdef __cplusplus
}
#endif

#endif /* AMOEBA_H */
