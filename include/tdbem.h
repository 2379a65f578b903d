/*
 * tdbem.h -- C ABI of the MI355X time-domain CFIE boundary element library.
 *
 * Operation (T. Takahashi, "A fast time-domain boundary element method for
 * three-dimensional electromagnetic scattering problems"):
 *   The induced current J = n x H (n the inward normal) on a perfectly
 *   conducting closed surface solves the CFIE  dL/dt(J) + theta eta (dK/dt(J) +
 *   zeta K(J)) = tested incident field  (Section 2.1, Eq. cfie), discretised with
 *   RWG bases in space and quadratic B-splines in time (Section 2.2) and
 *   Galerkin-tested (Section 2.4).  Marching on in time (Section 2.5, Eqs. solve
 *   and R) each step alpha solves
 *       Zt^(1) J^{alpha-1} = V^{alpha-1} - sum_{g>=2} Zt^(g) J^{alpha-g},
 *   where Zt^(g) are the coefficient matrices in the J-form (the paper's Jhat
 *   form of Eq. layer_disc summed by parts; the MFIE identity term 1/2 J adds
 *   1/2 theta eta Gram (1/dt + zeta/2) at g = 1 and (-1/dt + zeta/2) at g = 2).
 *   In IFMM mode the history sum is split into near pairs (exact coefficients,
 *   Program 2) and far pairs evaluated with the space-time interpolation-based
 *   FMM (Section 3: P2M/M2L/L2P of Eqs. ddotA_M, ddotA_fmm, dotphi_fmm, P_fmm,
 *   eval; M2M/L2L by re-interpolation; time gating of Programs 3-4).
 *
 * Conventions
 *   Units are SI.  Every [N_e] array at this interface is in the canonical
 *   RWG edge order: edges sorted lexicographically by (lo, hi) vertex index;
 *   T+ is the triangle whose counter-clockwise (outward) vertex order runs
 *   lo -> hi, T- the one running hi -> lo.  Batched arrays are [rhs][N_e]
 *   (edge index fastest).  Device pointers are HIP device memory on the
 *   current device; all work is stream-ordered on the stream given at setup.
 *
 * Ownership and errors
 *   The caller owns every buffer it passes; the library copies the mesh and
 *   never frees caller memory.  The context owns all device memory it
 *   allocates and releases it in tdbem_destroy.  Every function returns 0 on
 *   success or a negative TDBEM_E* code; tdbem_last_error() returns a
 *   thread-local message for the last failure.  A context is not thread-safe.
 */
#ifndef TDBEM_H
#define TDBEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    TDBEM_OK = 0,
    TDBEM_EINVAL = -1,      /* invalid argument, mesh or configuration */
    TDBEM_ENOMEM = -2,      /* device or host allocation failed */
    TDBEM_EHIP = -3,        /* a HIP runtime call failed */
    TDBEM_EBREAKDOWN = -4,  /* time hierarchy breaks down: no step per finest interval (M_t = 0, Remark 1 of Section 3.4.1) */
    TDBEM_ENOCONV = -5,     /* GMRES did not reach the tolerance within the iteration cap (Section 2.5) */
    TDBEM_EUNSTABLE = -6    /* late-time growth of the current beyond cfg.growth_limit (Section 4.3) */
};

enum { TDBEM_MODE_DIRECT = 0, TDBEM_MODE_IFMM = 1 };
/* Precision forms of the history evaluation (the Z0 solve, the current and
 * the right-hand side are FP64 in every form).  FP64: everything FP64.  FP32:
 * near-field coefficients stored in FP32, M2L operator and products in FP32 on
 * the matrix cores (moments and local expansions FP64).  BF16: near-field
 * coefficients stored in bf16 (FP64 sums), the FP32 M2L (the bf16 matrix-core
 * M2L is TDBEM_M2L_BF16).  The far field applies the
 * undifferentiated kernels to differenced currents; the window's terms cancel
 * down to the retarded potential, which amplifies rounding by about (window
 * steps)^2: the reduced forms are options whose error is measured. */
enum { TDBEM_FP64 = 0, TDBEM_FP32 = 1, TDBEM_BF16 = 2 };
/* Interpolants on p equispaced nodes (Section 3.2).  LAGRANGE: Lagrange
 * polynomials in space and time.  CHI_TIME: Lagrange in space; in time the
 * piecewise cubic Hermite interpolant whose node slopes are finite differences
 * of the node values (central inside, second-order one-sided at the ends), the
 * interpolant of the paper's earlier work; it reproduces quadratics and keeps
 * the late-time march stable where the Lagrange variant is not. */
enum { TDBEM_INTERP_LAGRANGE = 0, TDBEM_INTERP_CHI_TIME = 1 };
enum { TDBEM_GUESS_EXTRAP = 0, TDBEM_GUESS_LEARNED = 1 };
/* The CFIE (Section 2.1, Eq. cfie; variants of Section 4.3.1):
 *   CFIE1 = dt EFIE + theta eta (dt MFIE + zeta MFIE)   (the paper's choice),
 *   CFIE2 = dt EFIE + theta eta dt MFIE,
 *   CFIE3 = dt EFIE + theta eta zeta MFIE.
 * The variant weights every term of the MFIE's time derivative (kernel, the
 * identity term, the incident magnetic field) and of the MFIE itself. */
enum { TDBEM_CFIE1 = 1, TDBEM_CFIE2 = 2, TDBEM_CFIE3 = 3 };
/* Where the far field puts the second time derivative of the vector potential
 * (Section 4.3.2): SPLIT differentiates kernel and target interpolant once
 * each (dU/dt with l_m', Eq. ddotA_fmm, the paper's choice); KERNEL
 * interpolates d^2U/dt^2 = c^2 d (d - 1) U^{d-2} (with l_m); INTERP
 * interpolates U and differentiates the interpolant twice (l_m''). */
enum { TDBEM_DT2_SPLIT = 0, TDBEM_DT2_KERNEL = 1, TDBEM_DT2_INTERP = 2 };
/* M2L kernels (Section 3.6.1): AUTO, the operator tables of p = 4 in LDS on the
 * matrix cores (and the generic kernel for p = 6, 8); GENERIC, the dense M2L
 * for any p with the operator entries formed per lane from lattice distances
 * (the same products; slower at p = 4, where it checks the tuned kernel); FFT,
 * the M2L as a 4-D convolution evaluated in the Fourier domain (the node
 * lattice makes every operator a function of node-index differences, Section
 * 3.6.1, last paragraph): transformed kernels per offset and lag are set up
 * once, each interval's moments are transformed once, products are diagonal.
 * FFT computes in FP64 (precision must be TDBEM_FP64) and holds (2p)^3 (p+1)
 * complex values per moment vector (20x the dense moments at p = 4).  BF16
 * (p = 4): the tuned kernels with operator and moments rounded to bf16 on the
 * 16x16x32 bf16 matrix-core instruction, FP32 accumulation, whatever the
 * precision form; the far field's cancellation (window terms that grow with
 * the square of the lag) amplifies its rounding to errors of order one, so it
 * is a measured option, not an accurate one. */
enum { TDBEM_M2L_AUTO = 0, TDBEM_M2L_GENERIC = 1, TDBEM_M2L_FFT = 2, TDBEM_M2L_BF16 = 3 };
/* Z0 solver (Section 2.5): DEVICE, one cooperative kernel per step for every
 * right-hand side; HOST, the same GMRES driven from the host (reference). */
enum { TDBEM_SOLVER_DEVICE = 0, TDBEM_SOLVER_HOST = 1 };

typedef struct tdbem_ctx tdbem_ctx;

/* Closed, consistently (outward) oriented, manifold triangle mesh. */
typedef struct {
    int64_t n_vertices;
    const double *xyz;        /* host [n_vertices][3], metres; copied */
    int64_t n_triangles;
    const int32_t *tri;       /* host [n_triangles][3], counter-clockwise seen from outside */
} tdbem_mesh;

/* Configuration.  A zero-initialised struct is not valid: dt, eps, mu,
 * n_quad, n_rhs and the solver fields must be set (the Python binding gives
 * the paper's defaults). */
typedef struct {
    /* time discretisation (Section 2.2) */
    double dt;                /* time step [s] */
    int32_t nt;               /* number of time steps the context may march */
    int32_t d;                /* temporal B-spline order; must be 2 */
    /* medium and equation (Section 2.1) */
    double eps, mu;           /* permittivity [F/m], permeability [H/m] */
    double theta, zeta;       /* CFIE coupling constants (zeta in 1/s) */
    int32_t cfie;             /* TDBEM_CFIE1 | TDBEM_CFIE2 | TDBEM_CFIE3 */
    /* testing (Section 2.4) */
    int32_t n_quad;           /* points of the triangle rule of testing and of the far-field weights: 3 */
    /* far field (Section 3; IFMM mode) */
    int32_t p_s, p_t;         /* interpolation points per axis in space and in time: p_s = p_t = 4, 6 or 8
                                 (FAST4/6/8 of Section 4.2) */
    int32_t interp;           /* TDBEM_INTERP_LAGRANGE or TDBEM_INTERP_CHI_TIME */
    int32_t dt2;              /* TDBEM_DT2_SPLIT | TDBEM_DT2_KERNEL | TDBEM_DT2_INTERP */
    int32_t m2l;              /* TDBEM_M2L_AUTO | TDBEM_M2L_GENERIC | TDBEM_M2L_FFT | TDBEM_M2L_BF16 */
    int32_t leaf_max;         /* subdivide a cell while it holds more edges than this (Section 3.4.1) */
    int32_t min_level;        /* subdivide at least down to this level (2) */
    int32_t mu_window;        /* future intervals of the M2L (paper: 8, Section 3.6.1); raised if needed */
    int32_t box_widen;        /* 1: interpolation boxes = cells widened by the largest per-axis reach of a
                                 basis support beyond its edge midpoint (no extrapolation of the
                                 interpolants; for bodies whose finest cells are not much larger than their
                                 edges, e.g. structured cubes); 0: the cells (the paper) */
    int32_t causal_guard;     /* 1: steps per interval from the cell side minus twice that reach, so that no
                                 far pair interacts within one interval; 0: the cell side (Remark 1) */
    /* method and batch */
    int32_t mode;             /* TDBEM_MODE_DIRECT (all pairs exact) or TDBEM_MODE_IFMM */
    int32_t precision;        /* TDBEM_FP64 | TDBEM_FP32 | TDBEM_BF16 for near-field and M2L sums */
    int32_t n_rhs;            /* independent incident fields marched together */
    /* Z0 solve (Section 2.5) */
    double gmres_rtol;        /* relative residual tolerance */
    int32_t gmres_maxit;      /* Krylov iterations per step (cap) */
    int32_t gmres_restart;    /* Krylov vectors per restart cycle, 1..32 */
    int32_t guess;            /* TDBEM_GUESS_EXTRAP (quadratic extrapolation) or _LEARNED */
    int32_t solver;           /* TDBEM_SOLVER_DEVICE or TDBEM_SOLVER_HOST */
    int32_t gmres_blocks;     /* blocks per system of the device solve (0: automatic) */
    int32_t autotune;         /* 1: at set-up, time the near-field kernel's round shapes (lag steps and pair
                                 blocks per round) and, for one right-hand side with gmres_blocks = 0, the
                                 device solve's blocks per system, and keep the fastest (TDBEM_Q_TUNED);
                                 0: the fixed defaults */
    int32_t near_kernel;      /* near-field kernel: 0 the default (or the autotuner's choice); k >= 1 forces
                                 form k - 1.  One rhs: 0-4 the row kernel (each row's source currents
                                 gathered from the ring) with (lag steps, pair blocks) per round (2,1)
                                 (1,1) (3,1) (2,2) (1,2); 5-6 the per-leaf kernel (per chunk of a leaf's
                                 rows, the sources' currents staged in LDS) with 2 or 1 lag steps and 2
                                 pair blocks per round, the default (form 5) when any leaf's window fits.
                                 Several rhs: 0 the row kernel (lanes are right-hand sides); 7 the
                                 per-leaf matrix-core form (each leaf's coefficients as a dense block over
                                 its window: per source the lags its strips reach; multiplied by the
                                 sources' currents at those lags on the matrix cores; FP64 and FP32 forms),
                                 the default when it is built */
    int32_t graph;            /* 1: tdbem_march issues each step's kernels before and after the device solve
                                 as launches of HIP graphs captured from them (one graph for the kernels
                                 before the solve, one per pattern of far-field levels passing their time
                                 gate after it; later steps update the captured graphs' arguments).  The
                                 solve's cooperative launch stays a plain launch between the two.  Only
                                 with the device solver and while phase timing is off; the results are
                                 bitwise those of 0, the plain launches */
    /* late-time stability monitor (Section 4.3): 0 disables.  Once the tested
     * incident field of a right-hand side has fallen below 1e-6 of its largest
     * norm so far (the excitation has passed), a step returns TDBEM_EUNSTABLE
     * when the norm of that right-hand side's current exceeds growth_limit
     * times the largest current norm seen while the excitation lasted. */
    double growth_limit;
    void *stream;             /* hipStream_t for all work (NULL: the default stream) */
} tdbem_config;

/* Build the space-time hierarchy, the near-field J-form coefficients (computed
 * on the device, FP64 semi-analytic inner integrals, 3-point testing), the Z0
 * matrix and, in IFMM mode, the interpolation tables and M2L node values
 * (Sections 2.3-2.5 and 3.4.1).  On success *out receives a new context.
 * Errors: TDBEM_EINVAL (bad mesh/config, or an option not implemented:
 * p_s = p_t in {4, 6, 8} and n_quad = 3 only), TDBEM_EBREAKDOWN (no step per finest
 * interval, Remark 1 of Section 3.4.1, or a far-field window of more than 20
 * intervals), TDBEM_ENOMEM, TDBEM_EHIP. */
int tdbem_setup(const tdbem_mesh *mesh, const tdbem_config *cfg, tdbem_ctx **out);

/* Tested incident field V^{step-1} (Eq. v_i) of n_rhs plane-wave pulses at
 * t = step dt, written to V_dev [n_rhs][N_e] (device).  pulses: host array
 * [n_rhs][11] = k(3), polarisation(3), E0, f0, sigma, delay, kind (0 modulated
 * Gaussian cos(2 pi f0 tau) exp(-tau^2/2 sigma^2), 1 Sin^2 pulse of Section
 * 4.1, 2 Gaussian of Section 4.3), tau = t - delay - k.x/c. */
int tdbem_incident_planewave(tdbem_ctx *ctx, const double *pulses, int32_t step, double *V_dev);

/* Stateless history evaluation.  hist_dev [n_hist][n_rhs][N_e] (device) holds
 * J^0 .. J^{n_hist-1}; out_dev [n_rhs][N_e] (device) receives the history part
 * of the right-hand side of step alpha = n_hist + 1:
 *     sum_{g>=2} Zt^(g) J^{alpha-g}  (near pairs exact; far pairs by the IFMM
 * replayed over the whole history in IFMM mode).  Resets the marching state. */
int tdbem_potentials(tdbem_ctx *ctx, const double *hist_dev, int32_t n_hist, double *out_dev);

/* One marching step: V_dev [n_rhs][N_e] = V^{alpha-1} in, J_dev [n_rhs][N_e] =
 * J^{alpha-1} out (device); advances alpha.  TDBEM_ENOCONV if the Z0 solve
 * misses the tolerance (the iterate is still returned). */
int tdbem_step(tdbem_ctx *ctx, const double *V_dev, double *J_dev);

/* n_steps MOT steps in a row (Program 1), the same as n_steps calls of
 * tdbem_step, without a host wait between them: each step's GMRES status (and
 * the stability monitor's norms) stays on the device and is read once after
 * the last step, so the host enqueues the next step while the GPU works.
 * V_dev [n_steps][n_rhs][N_e] device, the tested incident fields of the steps
 * alpha .. alpha + n_steps - 1 (read only); J_dev [n_steps][n_rhs][N_e] device,
 * receives the currents.  status (host int32 [n_steps], may be NULL) receives
 * each step's code (TDBEM_OK, TDBEM_ENOCONV, TDBEM_EUNSTABLE), iters (host
 * int32 [n_steps], may be NULL) its GMRES iterations (the largest over the
 * right-hand sides).  Returns the
 * first non-OK step code, TDBEM_EHIP if a grid-barrier wait timed out.  Every
 * step runs (a step that did not converge keeps its last iterate, as
 * tdbem_step does).  The per-step records are device memory of the context,
 * grown on demand (16 n_rhs + 16 n_rhs bytes per step).  With the host-driven
 * solver the steps are taken one at a time. */
int tdbem_march(tdbem_ctx *ctx, const double *V_dev, double *J_dev, int32_t n_steps, int32_t *status,
                int32_t *iters);

/* For callers that cannot allocate device memory during the march (code under
 * graph capture, serving loops, harnesses that forbid allocation): the same
 * step as tdbem_step, with the Z0 solve's workspace (Krylov vectors, partial
 * sums, status and grid-barrier words) taken from a static 16 MiB array of the
 * library instead of the context; nothing is allocated by the call.  Limit:
 * n_rhs (35 N_e + 16896) + 2 N_e n_rhs [n_rhs > 1] + 1024 n_rhs + 2 n_rhs doubles
 * <= 2^21 (about N_e n_rhs <= 55000); beyond it TDBEM_EINVAL.  The array is
 * shared by every context on a device and keeps the last call's contents:
 * calls that overlap on one device race.  Needs the device solver
 * (TDBEM_SOLVER_DEVICE); with phase timing on (tdbem_profile) the timing
 * events are still created on first use.  The size check comes before any
 * work: a refused call leaves the context unchanged. */
int tdbem_step_noalloc(tdbem_ctx *ctx, const double *V_dev, double *J_dev);

/* Restart the march at alpha = 1 with zero history. */
int tdbem_reset(tdbem_ctx *ctx);

/* Checkpoint of the marching state (Program 1: what one step hands to the
 * next): the step counter, the ring of past currents, and in IFMM mode the
 * moments, local expansions, pending L2L contributions and far-field
 * potentials of every level (Programs 3-4), plus the stability monitor's
 * running norms.  Nothing setup derives from the mesh and configuration is
 * included.  buf NULL: *len receives the size in bytes.  Otherwise buf (host
 * memory of at least *len bytes, owned by the caller) receives the state and
 * *len its size; EINVAL if *len is too small.  Waits for the stream. */
int tdbem_checkpoint(const tdbem_ctx *ctx, void *buf, size_t *len);

/* Restore a checkpoint into a context set up from the same mesh and
 * configuration (the checkpoint records the sizes and a fingerprint of both;
 * EINVAL if they differ or the buffer is malformed).  The march then
 * continues bitwise as the checkpointed context would have.  buf: host
 * memory of len bytes, read only. */
int tdbem_restore(tdbem_ctx *ctx, const void *buf, size_t len);

enum {
    TDBEM_Q_NE = 0,          /* int64: number of edges */
    TDBEM_Q_EDGES = 1,       /* int32 [N_e][2]: (lo, hi) vertex ids in canonical order */
    TDBEM_Q_LMAX = 2,        /* int32: deepest octree level */
    TDBEM_Q_MT = 3,          /* int32 [l_max+1]: steps per interval per level (0 above level 2) */
    TDBEM_Q_NEAR_NNZ = 4,    /* int64: stored near-field coefficients (g >= 2) */
    TDBEM_Q_NEAR_PAIRS = 5,  /* int64: near (i, j) pairs */
    TDBEM_Q_Z0_NNZ = 6,      /* int64: non-zeros of Zt^(1) */
    TDBEM_Q_NCELLS = 7,      /* int32 [l_max+1]: cells per level */
    TDBEM_Q_NILIST = 8,      /* int64 [l_max+1]: interaction-list entries per level */
    TDBEM_Q_WINDOW = 9,      /* int32: largest number of far-field source intervals per M2L over the levels */
    TDBEM_Q_GMRES_ITERS = 10,/* int32: Krylov iterations of the last step (max over rhs) */
    TDBEM_Q_DEVICE_BYTES = 11,/* int64: device memory held by the context */
    TDBEM_Q_STEP = 12,       /* int32: next step alpha */
    TDBEM_Q_EDGE_LEAF = 13,  /* int32 [N_e]: internal (leaf-order) position of each canonical edge */
    TDBEM_Q_SETUP_MS = 14,   /* double: wall time of tdbem_setup */
    TDBEM_Q_PHASE_MS = 15,   /* double [TDBEM_NPHASE]: device time per phase since profiling was enabled */
    TDBEM_Q_PHASE_COUNT = 16, /* int64 [TDBEM_NPHASE]: timed launches per phase */
    TDBEM_Q_GUESS_USED = 17, /* int64: (step, rhs) pairs whose solve started from the learned guess */
    TDBEM_Q_CONFIG = 18,     /* tdbem_config: the configuration as set up (the switches in effect) */
    TDBEM_Q_D0_NNZ = 19,     /* int64: non-zero coefficients (i, j, g >= 1) of the discretised problem over
                                all pairs (the exact lag support of every pair, as the direct mode stores
                                it); computed on the device at the first query */
    TDBEM_Q_UNSTABLE = 20,   /* int32 [n_rhs]: 1 where the stability monitor has tripped */
    TDBEM_Q_WINDOWS = 21,    /* int32 [l_max+1]: source intervals per M2L per level, mu + ceil(3 / M_t(l)) (0 above
                                level 2): the window's oldest ceil(3 / M_t) intervals use differences truncated at
                                the oldest interval's start */
    TDBEM_Q_TUNED = 22,      /* int32 [4]: the near-field form in use (lag steps of 4 lags per round, 64-pair
                                blocks per round; 0 blocks: the per-leaf kernel; 0, 0: the batched
                                matrix-core form), the device solve's blocks per system (0: automatic) and 1
                                if the set-up autotuner chose them */
    TDBEM_Q_NEAR_LEAF_BYTES = 23, /* int64: device bytes of the dense per-leaf near-field blocks of the batched
                                matrix-core form (0 when they are not built: one rhs, the BF16 form, or over
                                the 32 GB limit) */
    TDBEM_Q_GRAPHS = 24      /* int64 [2]: executable graphs instantiated and argument refreshes by
                                tdbem_march with graph = 1 since set-up */
};

/* Phases timed by tdbem_profile (HIP events on the work stream around each
 * phase's launches).  TDBEM_PH_M2L times the M2L product kernel alone (one
 * launch per level and time gate); TDBEM_PH_M2L_SUM the per-target sum of its
 * interaction-list contributions (one right-hand side only). */
enum {
    TDBEM_PH_NEAR = 0, TDBEM_PH_GMRES = 1, TDBEM_PH_P2M = 2, TDBEM_PH_M2M = 3, TDBEM_PH_M2L = 4,
    TDBEM_PH_L2L = 5, TDBEM_PH_L2P = 6, TDBEM_PH_OTHER = 7, TDBEM_PH_M2L_SUM = 8, TDBEM_NPHASE = 9
};
int tdbem_query(const tdbem_ctx *ctx, int32_t key, void *out);

/* Near-field coefficients of chosen rows (for tests): rows [n] canonical edge
 * ids (host); out host [n][N_e][G] receives Zt^(g)_{row, j}, g = 0..G-1, for
 * every stored near pair (zero elsewhere, g = 1 included). */
int tdbem_near_rows(tdbem_ctx *ctx, const int32_t *rows, int32_t n, int32_t G, double *out);

/* Enable (1) or disable (0) per-phase timing; enabling clears the counters.
 * Timing synchronises nothing until a TDBEM_Q_PHASE_* query, which waits for
 * the stream and folds the recorded event pairs into the totals. */
int tdbem_profile(tdbem_ctx *ctx, int32_t enable);

/* Learned initial guess of the Z0 solve (not part of the paper's method: an
 * alternative to starting the solve of Eq. solve from the quadratic
 * extrapolation 3J^{a-2} - 3J^{a-3} + J^{a-4}).  Per edge i and right-hand side,
 * 116 features are formed:
 *   f = 8e + s - 1 (e = 0..12, s = 1..8): sigma_ie J_e^{alpha-1-s}
 *   f = 104 + e    (e = 0..11):           sigma_ie (R_e^{alpha-1} - (Z0 x)_e) / Z0_ee
 * with e = 0 the edge itself and e = 1..12 its 12 nearest edges by midpoint
 * distance (ties by canonical index), sigma_ie the sign of the dot product of
 * the two edges' T+ -> T- centroid directions, R the step's right-hand side
 * (V minus the near and far history) and x the extrapolation.  The features are divided by their
 * largest magnitude s_i (1 if all vanish) and rounded to bf16 (x).  With
 *   o(x) = relu(relu(x W1 + b1) W2 + b2) . w3 + b3
 * (W1, W2 and the hidden layer rounded to bf16, FP32 accumulation) the guess is
 *   J_guess = extrapolation + s_i (o(x) - o(-x)) / 2.
 * The solve starts from whichever of this guess and the extrapolation has the
 * smaller residual norm ||R - Z0 x|| (per right-hand side); it stays FP64 and
 * converges to the same tolerance from either. */
#define TDBEM_GUESS_NFEAT 116
#define TDBEM_GUESS_NHIDDEN 128
#define TDBEM_GUESS_NPARAMS (116 * 128 + 128 + 128 * 128 + 128 + 128 + 1)

/* Load the network: params host FP32 [TDBEM_GUESS_NPARAMS] in the order
 * W1 [116][128] (feature, hidden unit), b1 [128], W2 [128][128] (input unit,
 * output unit), b2 [128], w3 [128], b3.  Copied; EINVAL if n_params differs or a
 * value is not finite.  Steps of a context configured with
 * guess = TDBEM_GUESS_LEARNED fail with EINVAL until parameters are loaded. */
int tdbem_guess_weights(tdbem_ctx *ctx, const float *params, int64_t n_params);

/* Capture the guess inputs of the following steps (training data): before each
 * solve, features_dev (device FP32 [n_rhs][N_e][116], canonical edge order)
 * receives the normalised features x and aux_dev (device FP64 [n_rhs][N_e][2])
 * the scale s_i and the extrapolation.  The buffers are overwritten by every
 * step until capture is switched off with two null pointers; the caller owns
 * them and keeps them alive meanwhile. */
int tdbem_guess_capture(tdbem_ctx *ctx, float *features_dev, double *aux_dev);

/* Training of the guess network (FP32, no context needed).  Gradient of the
 * loss L = (1/n) sum_s (g(x_s) - y_s)^2 with g the odd network above evaluated
 * in FP32 without the bf16 roundings of inference:
 *   params_dev FP32 [TDBEM_GUESS_NPARAMS] (order of tdbem_guess_weights),
 *   X_dev FP32 [n][116] features, Y_dev FP32 [n] targets (the correction
 *   (J - extrapolation) / s of captured steps),
 *   grad_dev FP32 [TDBEM_GUESS_NPARAMS] receives dL/dparams (overwritten),
 *   loss_dev FP32 [1] receives L (overwritten).
 * All pointers are device memory owned by the caller; the work is issued on
 * stream (a hipStream_t; null for the default stream) and not waited for.
 * Gradient sums use atomic additions, so their rounding order varies. */
int tdbem_guess_grad(const float *params_dev, const float *X_dev, const float *Y_dev, int64_t n,
                     float *grad_dev, float *loss_dev, void *stream);

/* One Adam step in place on params_dev with moments m_dev, v_dev (device FP32
 * [TDBEM_GUESS_NPARAMS], zero before the first step) and step count t >= 1:
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
int tdbem_guess_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int32_t t,
                     float lr, float beta1, float beta2, float eps, void *stream);

void tdbem_destroy(tdbem_ctx *ctx);
const char *tdbem_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TDBEM_H */
