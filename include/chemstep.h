/*
 * chemstep.h -- C ABI of the MI355X per-cell chemistry-step library.
 *
 * The library advances the thermochemical state of many independent CFD cells
 * through one chemistry time step, the operation that the GPU-ANN method of
 * arXiv 2312.05800 moves onto the GPU (Sec. 2: the whole step stays on the
 * device, so no host/device copies happen inside it; Sec. 3.1: each
 * composition is integrated over the chemistry time step; Sec. 3.2: the ANN
 * maps {T, p, F(Y)} to the change of Y over the step).
 *
 * Conventions for every call below
 *   - Pointers are DEVICE pointers unless marked (host).
 *   - Cell arrays are SoA: scalar fields are [n] (element i at [i]); species
 *     fields are [K][ld] (species k of cell i at [k*ld + i]); ld >= n.
 *   - Units are SI: T in K, p in Pa, mass fractions dimensionless, rates in
 *     kg/m^3/s or mol/m^3/s as stated.
 *   - Calls are asynchronous and stream-ordered: `stream` is a hipStream_t
 *     passed as void* (NULL = the legacy default stream).  Argument errors are
 *     detected on the host before anything is launched and return an error
 *     code; the call then has no effect.  Per-cell numerical outcomes go to
 *     the per-cell stats/flags arrays, never to the return code.
 *   - The caller owns every cell array.  Handles own their device copies of
 *     constants, weights and workspace.  Calls that use the same handle
 *     concurrently on different streams race on its workspace and must be
 *     ordered by the caller.
 *   - The library never exits or aborts.  A failed HIP call returns
 *     CHEM_EHIP with the HIP error text in chem_last_error().
 */
#ifndef CHEMSTEP_H
#define CHEMSTEP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CHEM_OK = 0,
  CHEM_EINVAL = 1,       /* bad argument (null pointer, size, ld < n, ...) */
  CHEM_ENOMEM = 2,       /* device allocation failed */
  CHEM_EHIP = 3,         /* a HIP runtime call failed */
  CHEM_EMECH = 4,        /* inconsistent mechanism description */
  CHEM_EMODEL = 5,       /* inconsistent network / model file */
  CHEM_EUNSUPPORTED = 6  /* valid but beyond the library's limits (e.g. K > 63) */
} chem_status;

/* Per-cell status codes written to stats[2][i] by chem_step. */
enum {
  CHEM_CELL_OK = 0,
  CHEM_CELL_MAX_STEPS = 1,   /* more than max_steps step attempts */
  CHEM_CELL_H_UNDERFLOW = 2, /* step size fell below h_min */
  CHEM_CELL_NONFINITE = 3,   /* non-finite input state, or T <= 0, or p <= 0 */
  CHEM_CELL_SINGULAR = 4     /* zero or non-finite pivot in the Newton matrix */
};

/* Human-readable name of a status code (static string). */
const char *chem_status_string(chem_status s);
/* Detail of the last error on the calling host thread (thread-local). */
const char *chem_last_error(void);

/* ------------------------------------------------------------ mechanism
 * A reaction mechanism: K species over E elements, R reversible elementary
 * reactions (one or two reactant and product species, stoichiometric
 * coefficients 1 or 2, no third bodies).  Thermo per species is NASA-7
 * (low range for T <= T_mid, else high range); forward rate constants are
 * k_f = A T^b exp(-Ea/(R T)); reverse ones k_f/K_c with K_c from the standard
 * Gibbs energies at p_ref = 101325 Pa.  All pointers in the descriptor are
 * (host) and are copied at create time. */
typedef struct {
  int32_t K, R, E;
  const double *W;       /* (host) [K] molar mass, kg/mol */
  const int32_t *comp;   /* (host) [K][E] atoms of element e in species k */
  const double *awt;     /* (host) [E] atomic weight, kg/mol */
  const double *nasa;    /* (host) [K][17]: T_low, T_mid, T_high, low a1..a7, high a1..a7 */
  const int32_t *rsp;    /* (host) [R][4]: reactant0, reactant1, product0, product1; -1 = none */
  const int32_t *rnu;    /* (host) [R][4]: stoichiometric coefficient (1 or 2) of each slot */
  const double *A;       /* (host) [R] SI: (m^3/mol)^(order-1)/s */
  const double *b;       /* (host) [R] temperature exponent */
  const double *Ea;      /* (host) [R] activation energy, J/mol */
} chem_mech_desc;

typedef struct chem_mech chem_mech;

/* Validate `desc` (element balance of every reaction, index ranges, K <= 63,
 * finite positive A and W) and upload it.  On success *out owns device memory
 * until chem_mech_destroy.  Errors: CHEM_EINVAL (null), CHEM_EMECH
 * (inconsistent), CHEM_EUNSUPPORTED (too large), CHEM_ENOMEM, CHEM_EHIP. */
chem_status chem_mech_create(const chem_mech_desc *desc, chem_mech **out);
void chem_mech_destroy(chem_mech *m);
int32_t chem_mech_num_species(const chem_mech *m);
int32_t chem_mech_num_reactions(const chem_mech *m);

typedef struct {
  int64_t n;   /* number of cells (0 is allowed: the call does nothing) */
  int64_t ld;  /* leading dimension of [K][ld] arrays, >= n */
} chem_batch;

/* Integrator controls; NULL selects the defaults in brackets.
 *   rtol [1e-6], atol_Y [1e-12], atol_T [1e-6 K]: error weights
 *       atol + rtol*max(|y_old|, |y_new|) per component;
 *   h0 [1e-8 s]: first step when no hint is given; h_min [1e-20 s];
 *   max_steps [100000] step attempts per cell. */
typedef struct {
  double rtol, atol_Y, atol_T, h0, h_min;
  int32_t max_steps;
} chem_step_opts;

/* Instantaneous chemistry of each cell (the reaction-rate evaluation the
 * paper's ANN replaces, Sec. 1 and Sec. 3.2):
 *   wdot [K][ld] net molar production rate, mol/m^3/s;
 *   dTdt [n]     adiabatic constant-pressure temperature rate, K/s (nullable);
 *   kfkr [2R][ld] forward rate constants in rows 0..R-1, reverse in R..2R-1,
 *                 SI (nullable).
 * Inputs T [n], p [n], Y [K][ld] are read only. */
chem_status chem_rates(const chem_mech *m, chem_batch batch, const double *T, const double *p,
                       const double *Y, double *wdot, double *dTdt, double *kfkr, void *stream);

/* One chemistry step of every cell (Sec. 3.1: integrate each composition
 * over the time step): the adiabatic constant-pressure reactor
 *   dY_k/dt = W_k wdot_k / rho,  dT/dt = -sum_k h_k wdot_k / (rho c_p)
 * integrated over [0, dt] by the 4-stage L-stable Rosenbrock method RODAS3
 * with its analytic Jacobian, an embedded error estimate and adaptive step
 * size, in FP64.
 *   dt          step for every cell, s (> 0) unless dt_cell is given;
 *   dt_cell     [n] per-cell step, s (nullable);
 *   T  [n]      in/out temperature;  p [n] pressure (constant over the step);
 *   Y  [K][ld]  in/out mass fractions (not clipped: tiny negatives may occur);
 *   RR [K][ld]  out rho(T0, Y0) (Y - Y0) / dt, kg/m^3/s (nullable);
 *   h_hint [n]  in/out step-size hint; <= 0 means none (nullable);
 *   stats [3][ld] out int32 rows: accepted steps, rejected steps, CHEM_CELL_*
 *               status (nullable).
 * A failed cell keeps its input T and Y, gets RR = 0 and its status. */
chem_status chem_step(const chem_mech *m, chem_batch batch, double dt, const double *dt_cell,
                      double *T, const double *p, double *Y, double *RR, double *h_hint,
                      int32_t *stats, const chem_step_opts *opts, void *stream);

/* One set of cells of an uneven batched workload. */
typedef struct {
  int64_t n;        /* cells in the set (0 allowed) */
  int64_t ld;       /* leading dimension of the set's [K][ld] arrays, >= n */
  double dt;        /* chemistry time step of the set, s (> 0) */
  double *T;        /* [n] in/out */
  const double *p;  /* [n] */
  double *Y;        /* [K][ld] in/out */
  double *RR;       /* [K][ld] out, nullable */
  double *h_hint;   /* [n] in/out, nullable */
  int32_t *stats;   /* [3][ld] out, nullable */
} chem_set;

/* chem_step over several independent cell sets with their own dt in one
 * persistent launch: the cells of all sets share one work queue, so sets of
 * very different size and stiffness keep every wavefront busy.  `sets` is a
 * (host) array of n_sets descriptors whose pointers are device pointers; the
 * table is copied to device memory owned by `m` on `stream`, and the call
 * synchronises `stream` while it stages that copy (calls on the same handle
 * must be ordered by the caller).  Results per cell are those of chem_step
 * with the set's dt. */
chem_status chem_step_sets(const chem_mech *m, int32_t n_sets, const chem_set *sets,
                           const chem_step_opts *opts, void *stream);
/* chem_step_sets with the table of n_sets descriptors already in device
 * memory (`sets`: device array, its pointers device pointers), for callers
 * that keep the step on the GPU without host round trips (Sec. 2): the set
 * offsets and the cell count are formed on the device, the launch is a full
 * persistent grid whose waves stop at that count, and nothing synchronises.
 * A set with n < 0, ld < n, null T, p or Y, or a dt that is not finite and
 * positive is skipped (its arrays untouched) and counted in *n_bad (device
 * int32, nullable).  The handle keeps the offsets: the first call with more
 * sets than before allocates (and so cannot be captured), and calls on one
 * handle must be ordered.  Host-side errors: null handle or table, more than
 * 2^20 sets, invalid options. */
chem_status chem_step_sets_device(const chem_mech *m, int32_t n_sets, const chem_set *sets,
                                  const chem_step_opts *opts, int32_t *n_bad, void *stream);

/* ------------------------------------------------------------ surrogate
 * The ANN of Sec. 3.2 that stands in for the integration: inputs
 * x = {T, p, F(Y)} with the Box-Cox transform F(y) = (y^lambda - 1)/lambda
 * (lambda = 0.1; negative y clamped to 0), z-score normalised with training
 * statistics; three GELU hidden layers (1600, 800, 400 in the paper); a linear
 * output u, the z-scored change Y(t+dt) - Y(t) of the mass fractions (the
 * output is not transformed).  Hidden GEMMs run on
 * BF16 MFMA with FP32 accumulation.  Trained with the L1 loss (Eq. Loss) and
 * Adam on FP32 master weights. */
typedef struct ann_model ann_model;

typedef struct {
  int32_t n_in;       /* K + 2 for a mechanism with K species */
  int32_t n_out;      /* K */
  int32_t hidden[3];  /* hidden widths */
  int32_t prec;       /* 0 = BF16 everywhere (the only value the library accepts) */
  int32_t members;    /* 0 or 1: one network with n_out outputs; n_out: the per-species
                         ensemble of Sec. 3.2 (one network with the same inputs and hidden
                         widths and a single output per species; their loss is the mean of
                         the members' L1 losses).  Every entry point takes either; the
                         physics terms of the loss and the FP8 variant need one network. */
} ann_arch;

/* Normalisation and validity statistics (all arrays host, copied). */
typedef struct {
  float lambda;          /* Box-Cox exponent */
  double dt_model;       /* time step the network was trained for, s */
  const float *mu_in, *sd_in;   /* [n_in] input z-score */
  const float *lo, *hi;         /* [n_in] training range of the raw inputs (OOD test) */
  const float *mu_out, *sd_out; /* [n_out] output z-score */
} ann_norm;

/* New network with weights and biases ~ U(-1/sqrt(fan_in), 1/sqrt(fan_in))
 * from `seed`, zero Adam state, no statistics.  Owns device memory. */
chem_status ann_create(const ann_arch *arch, uint64_t seed, ann_model **out);
void ann_destroy(ann_model *m);
/* Layer l in 0..3: W (host) [out][in] row-major FP32, b (host) [out].  In an
 * ensemble, index 4 g + l is layer l of member g (its output layer has one
 * row). */
chem_status ann_set_layer(ann_model *m, int32_t layer, const float *W, const float *b);
chem_status ann_get_layer(const ann_model *m, int32_t layer, float *W, float *b);
/* Gradients of the loss from the last ann_train_step (host arrays as above). */
chem_status ann_get_grad(const ann_model *m, int32_t layer, float *dW, float *db);
/* Adam's first and second moments of layer l (host arrays as for the layer:
 * mW, vW [out][in], mb, vb [out]; any may be NULL): the optimiser state the
 * next ann_train_step continues from (Sec. 3.2, Adam). */
chem_status ann_get_moments(const ann_model *m, int32_t layer, float *mW, float *vW, float *mb,
                            float *vb);
chem_status ann_set_norm(ann_model *m, const ann_norm *norm);
/* Host copies of the statistics; any pointer may be NULL. */
chem_status ann_get_norm(const ann_model *m, float *mu_in, float *sd_in, float *lo, float *hi,
                         float *mu_out, float *sd_out, float *lambda, double *dt_model);
/* Statistics from a training set of n state pairs (Y1 = Y0 integrated over
 * dt_model): mean and population standard deviation (a zero spread becomes 1)
 * and range of every input feature and every target.  Synchronises `stream`. */
chem_status ann_fit_norm(ann_model *m, chem_batch batch, const double *T, const double *p,
                         const double *Y0, const double *Y1, float lambda, double dt_model,
                         void *stream);
/* Network output only: U [n][n_out] row-major FP32, z-space. */
chem_status ann_forward(ann_model *m, chem_batch batch, const double *T, const double *p,
                        const double *Y, float *U, void *stream);

typedef struct {
  float residual_tol;   /* [1e-6] max |element mass fraction change| allowed */
  float ood_margin;     /* [0.05] widening of the training range, fraction of its span */
  int32_t fallback;     /* [1] integrate flagged cells with chem_step */
  float audit_fraction; /* [0] share of the cells also integrated by chem_step to judge the
                           network (in [0, 1]; see ann_step) */
  double *audit;        /* device [3 + 3K] doubles, out: the audit (needed when
                           audit_fraction > 0, else ignored) */
} ann_step_opts;

/* The surrogate chemistry step of every cell (the ANN replacing the
 * reaction-rate integration, Sec. 1-2): Y' = Y0 + sd_out u + mu_out from
 * the network, projected onto element conservation by weighted least
 * squares (weight of species k: sd_out,k^2 (Y+_k + 1e-10) / (Y+_k + sd_out,k)
 * with Y+ = max(Y', 0): the expected variance of the network's error in its
 * change, tapered to zero as the species vanishes), clipped at 0; T from h(T, Y) = h(T0, Y0) by
 * FP64 Newton; RR = rho0 (Y - Y0)/dt.  A cell is flagged (flags [n], nullable)
 * with bit 0 if an input lies outside the widened training range or dt
 * differs from dt_model, bit 1 if the element residual of the network's own
 * state Y' (max_e |(M Y')_e - (M Y0)_e|, M the element mass fractions per
 * unit mass fraction) or of the projected state exceeds residual_tol;
 * flagged cells keep their input state and, with fallback on, are integrated
 * by chem_step (fb_opts) on the same stream without a host round trip; bit 2
 * marks a failed fallback.  n_fallback (device int64, nullable) receives the
 * number of flagged cells.  Workspace grows on the first call with a larger n.
 * Audit (the integrator judging the network inside the step): with
 * audit_fraction f > 0, every s-th cell (s the integer nearest 1/f; cells 0,
 * s, 2s, ... of the batch)
 * is also integrated from its input state by chem_step (fb_opts), and
 * opts->audit receives, for this call: [0] the audited cells the network
 * handled, [1] the audited cells not compared (flagged by the network, or
 * whose reference integration failed), [2] the largest |T - T_ref|, and per
 * species k: [3 + 3k] the sum over the compared cells of (Y_k - Y_ref,k)^2,
 * [4 + 3k] and [5 + 3k] the smallest and largest reference change
 * Y_ref,k - Y0,k (so that the normalised RMSE of species k is
 * sqrt([3 + 3k] / [0]) / ([5 + 3k] - [4 + 3k])).  The sums use atomics: their
 * last bits vary from run to run.  The audited cells' reference integration
 * is one more chem_step launch per chunk of cells. */
chem_status ann_step(ann_model *m, const chem_mech *mech, chem_batch batch, double dt, double *T,
                     const double *p, double *Y, double *RR, uint8_t *flags,
                     int64_t *n_fallback, const ann_step_opts *opts,
                     const chem_step_opts *fb_opts, void *stream);

/* ann_step for callers that cannot allocate device memory: code being
 * captured into a HIP graph, tight serving loops, harnesses that forbid
 * hipMalloc.  Same kernels, arguments, results and error behaviour as
 * ann_step, but the inference workspace and the fallback list live in a
 * file-scope device array of 64 MiB (one per GPU the library runs on, held
 * until the process ends); the call makes no hipMalloc, hipFree or other
 * allocating call.  All cells of a call must fit in it as one chunk: a
 * batch larger than the network's capacity (7 999 cells for the
 * 32-1600-800-400-30 network: 64 MiB over its 8.4 KB of per-cell
 * activations, E4M3 rows and fallback entry) is
 * rejected with CHEM_EINVAL, and chem_last_error() states the maximum.  The
 * model and the mechanism must be on the current device.  Calls on one GPU
 * share the array, so calls that overlap in time (other streams, other
 * threads) race; calls ordered on one stream do not.  The audit needs its
 * own workspace: audit_fraction must be 0 here. */
chem_status ann_step_noalloc(ann_model *m, const chem_mech *mech, chem_batch batch, double dt,
                             double *T, const double *p, double *Y, double *RR, uint8_t *flags,
                             int64_t *n_fallback, const ann_step_opts *opts,
                             const chem_step_opts *fb_opts, void *stream);

typedef struct {
  float lr, beta1, beta2, eps;
  /* weights of the physics terms of the loss (Sec. 3.2: mass-fraction sum,
   * energy and heat release rate); 0 leaves the L1 loss of Eq. (Loss) alone */
  float w_mass, w_energy, w_hrr;
} ann_train_opts;

/* One optimisation step on a batch of B state pairs (B a multiple of 32):
 * features and targets from T, p, Y0 and Y1 (Y0 integrated over dt_model),
 * gathered through index (device int64 [B], nullable: cells 0..B-1 with ld);
 * forward pass keeping activations; L1 loss (mean over samples and outputs,
 * Eq. (Loss)) written to *loss (device float); backward pass (BF16 operands,
 * FP32 accumulation, deterministic bias reductions); Adam with bias
 * correction on the FP32 master weights, refreshing the BF16 copies.  lr = 0
 * computes the gradients only (no update, step count unchanged).
 * Physics terms (Sec. 3.2 names the three principles, not their form; the
 * reading here): with dY = sd_out u + mu_out the predicted change and
 * e = (u - u*) sd_out its error, three L1 penalties |s_t| / D_t, averaged
 * over the batch: s = sum_k dY_k (the mass fractions keep summing to one),
 * s = sum_k h_k(T1) e_k (the state keeps the reference step's enthalpy at
 * its final temperature T1) and s = sum_k h_k(298.15 K) e_k (the heat
 * released over the step equals the reference's), h_k in J/kg from the
 * mechanism's NASA polynomials and D_t = sum_k |a_tk| sd_out,k the size of
 * the functional for errors of one standard deviation.  With any weight
 * non-zero or terms non-null, mech (the network's species) and T1 (device
 * [ld], gathered like T) are required, *loss becomes the L1 loss plus the
 * weighted terms and terms (device float [3], nullable) receives the three
 * unweighted batch means. */
chem_status ann_train_step(ann_model *m, const chem_mech *mech, chem_batch batch,
                           const double *T, const double *p, const double *Y0,
                           const double *Y1, const double *T1, const int64_t *index,
                           const ann_train_opts *opts, float *loss, float *terms, void *stream);
int64_t ann_num_steps(const ann_model *m);
/* Block and tile shapes of the training step, picked by measurement (the
 * step is launch- and latency-bound at training batches, so the best tiling
 * differs from the inference rule): each of the eleven products of a step at
 * batch B (forward, weight gradient and data gradient of every layer; an
 * ensemble's members grouped) is timed with every generic tiling (128 x 128,
 * 128 x 32, 64 x 64, 128 x 64 blocks; 32- or 64-wide K-steps) and, for the
 * weight gradients, every split along the batch the workspace holds (1..16),
 * on the model's training workspace; the fastest stays in the model for later
 * ann_train_step calls at batch B (other batches keep the built-in rules).
 * ms_default / ms_tuned (host, nullable) receive the summed product times
 * with the built-in rules and the chosen tilings.  With CHEM_AUTOTUNE_CACHE
 * naming a file, a result stored there for this device, network and batch
 * is taken without timing, and new results are stored.  Overwrites the last
 * step's gradients; synchronises `stream`. */
chem_status ann_autotune_train(ann_model *m, int64_t B, double *ms_default, double *ms_tuned,
                               void *stream);
/* FP8 variant of inference: the two hidden-to-hidden layers run on OCP FP8
 * E4M3 MFMA with per-tensor scales amax/448 -- activation scales from a BF16
 * forward pass over the calibration cells (at most 2^21 of them), weight
 * scales from the FP32 master weights; the first and last layers stay BF16.
 * Switches inference (ann_forward, ann_step) to FP8; synchronises `stream`.
 * A training step with lr > 0 switches back to BF16 (weights changed). */
chem_status ann_quantize_fp8(ann_model *m, chem_batch calib, const double *T, const double *p,
                             const double *Y, void *stream);
/* 0 = BF16 inference, 1 = FP8 hidden layers (requires ann_quantize_fp8). */
chem_status ann_set_precision(ann_model *m, int32_t prec);
/* Scales of the FP8 layers (host [2] each): activation and weight scale of
 * the 2nd and 3rd layer. */
chem_status ann_get_fp8_scales(const ann_model *m, float *act, float *wgt);
/* Binary model file: architecture, statistics, master weights, Adam state
 * (not the FP8 copies: quantise again after loading). */
chem_status ann_save(const ann_model *m, const char *path);
chem_status ann_load(const char *path, ann_model **out);

/* ------------------------------------------------------ launch autotuning
 * The persistent integrator's launch shape: lanes per cell (a power of two
 * >= K + 1, at most 64; a wavefront carries 64 / lanes cells) and resident
 * wavefronts per CU (each holds its cells' LDS slices; 0 = as many as the LDS
 * allows).  Per-cell results do not depend on the shape beyond the rounding
 * of wave-level reductions (well inside the step's error control). */
typedef struct {
  int32_t lanes_per_cell; /* 0 = the smallest power of two >= K + 1 */
  int32_t waves_per_cu;   /* 0 = LDS-limited maximum */
  double cells_per_s;     /* measured by chem_autotune (output only) */
} chem_tuning;

/* For the GPU chemistry step of Sec. 2 under uneven stiffness across cells:
 * times chem_step with every candidate launch shape on a device copy of the
 * sample cells (T, p, Y as in chem_step; the caller's arrays are not
 * modified), keeps the fastest in the mechanism handle for later chem_step,
 * chem_step_sets and fallback launches, and returns it (host, nullable).
 * Allocates and frees its scratch copies and synchronises `stream`; must not
 * run concurrently with other calls on the same handle.  With the environment
 * variable CHEM_AUTOTUNE_CACHE naming a file, a shape stored there for this
 * device, mechanism, dt and tolerances is applied without timing, and a new
 * measurement is stored ("key = value" text lines). */
chem_status chem_autotune(chem_mech *m, chem_batch sample, double dt, const double *T,
                          const double *p, const double *Y, const chem_step_opts *opts,
                          void *stream, chem_tuning *best);
/* Set the launch shape by hand (NULL = the default heuristic); CHEM_EINVAL for
 * a shape the mechanism cannot use. */
chem_status chem_set_tuning(chem_mech *m, const chem_tuning *t);
/* The launch shape chem_step will use (lanes_per_cell and waves_per_cu
 * resolved; cells_per_s as last measured, else 0). */
chem_status chem_get_tuning(const chem_mech *m, chem_tuning *out);

/* ------------------------------------------------------- captured steps
 * Sec. 2 keeps the whole time step on the GPU without host round trips; a
 * step recorded once as a HIP graph is replayed by one launch: the same
 * kernels, arguments and device pointers as the call that was captured (the
 * arrays are read and written again at every replay, so refill them between
 * replays).  Workspace growth happens before capture; afterwards the model's
 * inference workspace cannot grow (a larger ann_step returns CHEM_EINVAL)
 * until its graphs are destroyed.  Destroy every graph before the model or
 * mechanism it refers to. */
typedef struct chem_graph chem_graph;
/* ann_step captured; the BF16 weight layouts are rebuilt inside the graph, so
 * replays use the model's current weights (training between replays is
 * seen); precision and options are those at capture. */
chem_status ann_step_graph_create(ann_model *m, const chem_mech *mech, chem_batch batch,
                                  double dt, double *T, const double *p, double *Y, double *RR,
                                  uint8_t *flags, int64_t *n_fallback,
                                  const ann_step_opts *opts, const chem_step_opts *fb_opts,
                                  void *stream, chem_graph **out);
/* chem_step captured (launch shape as tuned at capture). */
chem_status chem_step_graph_create(const chem_mech *m, chem_batch batch, double dt,
                                   const double *dt_cell, double *T, const double *p, double *Y,
                                   double *RR, double *h_hint, int32_t *stats,
                                   const chem_step_opts *opts, void *stream, chem_graph **out);
/* chem_step_sets captured: the set table is validated and copied into
 * device memory owned by the graph (synchronising `stream`), so replays
 * integrate the same sets whatever later calls do. */
chem_status chem_step_sets_graph_create(const chem_mech *m, int32_t n_sets, const chem_set *sets,
                                        const chem_step_opts *opts, void *stream,
                                        chem_graph **out);
/* Replay on `stream` (asynchronous). */
chem_status chem_graph_launch(chem_graph *g, void *stream);
/* Destroy a graph whose replays have finished (synchronise their stream). */
void chem_graph_destroy(chem_graph *g);

/* ------------------------------------------------ training-set sampler */
/* Options of the training-set sampler.  Defaults of Sec. 3.1 and Table 1:
 * alpha 0.125, beta 10, gamma 0.1, T_min 500 K, H/C in [2.65, 4.67], O/N in
 * [0.254, 0.32], phi in [0.20, 1.15]. */
typedef struct {
  double alpha, beta, gamma; /* Eqs. (Trand)-(Yrand) */
  double T_min;              /* samples below are dropped */
  double hc_min, hc_max, on_min, on_max, phi_min, phi_max; /* Table 1 */
  int32_t n2;                /* species index of N2 */
  int32_t el_C, el_H, el_O, el_N; /* element indices of C, H, O, N */
} chem_sample_opts;

/* The random-data generation of the training set (Sec. 3.1), one sample per
 * seed i.  With s[i] < 0 (or s NULL) the seed (T, p, Y; SoA [K][ld], device)
 * is perturbed: T' = T + alpha c_T (T_max - T_min), p' = p + beta c_p
 * (p_max - p_min), y'_N2 = y_N2 + alpha c_N2 (y_N2,max - y_N2,min) with the
 * extremes over all n seeds, y'_j = y_j^(1 + gamma c_j) for every other
 * species with y_j > 0 (0 otherwise), and those species rescaled so that
 * the mass fractions sum to one.  With s[i] >= 0 the sample is the state
 * (1 - s) end_eq + s end_air on the line between two end states (device
 * [K + 2] each: T, p, Y_1..K; the paper's ends are the equilibrium of its
 * leanest mixture, phi = 0.45, and ambient air).  c: device [K + 3][ld]
 * random numbers in [-1, 1] (rows T, p, N2, then species j at row 3 + j).
 * keep[i] (device uint8 [n]) is 1 when the sample has T >= T_min, finite
 * non-negative mass fractions, and molar H/C, O/N and equivalence ratio
 * (2 n_C + n_H / 2) / n_O inside the limits.  Outputs T_out, p_out (device
 * [n]) and Y_out (device [K][ld]) are written for every sample.  Argument
 * errors are detected on the host; the first call allocates a small
 * range buffer owned by the mechanism handle. */
chem_status chem_sample_states(const chem_mech *m, chem_batch seeds, const double *T,
                               const double *p, const double *Y, const double *c,
                               const double *s, const double *end_eq, const double *end_air,
                               const chem_sample_opts *opts, double *T_out, double *p_out,
                               double *Y_out, uint8_t *keep, void *stream);

/* ------------------------------------------------- turbulence closure */
/* Options of the PaSR closure; NULL selects eta = 1e-3. */
typedef struct {
  double eta; /* a species takes part when |RR_k| >= eta max_j |RR_j| (in [0, 1]) */
} chem_pasr_opts;

/* Partially stirred reactor closure of the chemistry source (Sec. 4.1),
 * applied to the result of a step (chem_step or ann_step): every rate of a
 * cell is multiplied by its reacting fraction
 *   kappa = tau_c / (tau_c + tau_mix),  tau_mix = sqrt(tau_T tau_K),
 * where tau_T and tau_K are the flow solver's Taylor and Kolmogorov times and
 * tau_c is the slowest chemical time max_k rho Y_k / |RR_k| over the species
 * that take part (|RR_k| >= eta max_j |RR_j|, RR_k != 0), with rho the
 * ideal-gas density of (T, p, Y) and Y clipped at 0.  A cell without such a
 * species (all rates zero), or with tau_c + tau_mix = 0, has kappa = 1;
 * otherwise a negative or NaN product tau_T tau_K gives kappa = NaN.
 *   T [n], p [n]      state after the step (device, read);
 *   Y [K][ld]         mass fractions after the step (device, read);
 *   RR [K][ld]        in: the step's rates, kg/m^3/s; out: kappa RR (device);
 *   tau_taylor [n], tau_kolmogorov [n]  flow time scales, s (device, read);
 *   kappa [n], tau_c [n]  out (device, nullable; tau_c = +inf without a
 *                     reacting species).
 * One thread per cell, asynchronous on `stream`; argument errors (null
 * arrays, ld < n, eta outside [0, 1]) are detected on the host. */
chem_status chem_pasr_scale(const chem_mech *m, chem_batch batch, const double *T,
                            const double *p, const double *Y, double *RR,
                            const double *tau_taylor, const double *tau_kolmogorov,
                            const chem_pasr_opts *opts, double *kappa, double *tau_c,
                            void *stream);

/* Attainable peaks of this GPU, measured: dense BF16 MFMA, FP8 MFMA
 * (E4M3 operands, unit block scales) and FP64 vector FMA, each by a launch
 * of 2048 blocks of 256 threads running eight independent accumulator
 * chains per wave (one untimed warm-up launch first).  tflops (host [3])
 * receives TFLOP/s in that order.  Synchronises `stream`; allocates and frees
 * a small sink buffer. */
chem_status chem_measure_peaks(double *tflops, void *stream);

/* ---------------------------------------------------------- launch timing
 * Instrumentation for measurement: when enabled, every kernel launch the
 * library issues is bracketed by HIP events on its own stream.
 * chem_profile_read synchronises on those events and returns, per launch
 * label (host char[48]), the number of launches and their total duration in
 * milliseconds since the previous read; returns the number of labels written
 * (at most cap).  Off by default; costs two event records per launch. */
void chem_profile_enable(int32_t on);
int32_t chem_profile_read(char (*names)[48], int64_t *launches, double *total_ms, int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* CHEMSTEP_H */
