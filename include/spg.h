/*
 * spg.h - C ABI of the MI355X (gfx950) PEPS branch-and-bound hot path.
 *
 * The library finds low-energy states of a generalized Potts model (paper,
 * Sec. 2, Eq. (1)) on a rows x cols square or king's-graph lattice of clusters
 * (Fig. 1(b)): it builds the Boltzmann-weight PEPS (Fig. 1(c)), contracts it
 * row by row into boundary MPSs (Fig. 1(d)), and runs the branch-and-bound
 * (beam) search over conditional marginals (Fig. 1(d)-(e)).  Every step runs
 * in HIP kernels on the GPU; the host only validates arguments, sizes buffers
 * and enqueues work.
 *
 * Conventions shared by every entry point
 *   - Return value: SPG_OK (0) or a negative SPG_ERR_* code; the message of the
 *     last failure on the calling thread is returned by spg_last_error().
 *     Arguments are validated before anything is enqueued, so an error return
 *     leaves outputs untouched unless stated otherwise.
 *   - Streams: `stream` is a hipStream_t (NULL = the default stream).  Work is
 *     enqueued on it; a call blocks when it writes a HOST output, when it
 *     allocates device memory (allocation and its zero fill are
 *     device-synchronous: a new env, a first search on an env, larger beams),
 *     and spg_boundary_mps blocks until its contraction has finished (its
 *     workspace lives for the call).
 *   - Ownership: spg_peps_t and spg_env_t are library-owned and freed with
 *     their spg_free_* call.  Every buffer passed in is caller-owned; DEVICE
 *     pointers must stay valid until the enqueued work completes.
 *   - A handle is not thread-safe; an env keeps a pointer to its peps, which
 *     must outlive it.
 *   - Sites are numbered row-major, site = r * cols + c.  Local states are
 *     0 .. d-1.
 *   - Limits: 1 <= rows, 2 <= cols, 2 <= d <= 256, 1 <= chi <= 80,
 *     1 <= max_states <= 65536; larger values return SPG_ERR_UNSUPPORTED.
 */
#ifndef SPG_H
#define SPG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SPG_OK = 0,
  SPG_ERR_INVALID = -1,     /* bad argument (null pointer, inconsistent sizes)   */
  SPG_ERR_OOM = -2,         /* device allocation failed                          */
  SPG_ERR_HIP = -3,         /* a HIP runtime call failed                         */
  SPG_ERR_NONFINITE = -4,   /* non-finite energy, beta or log-scale              */
  SPG_ERR_UNSUPPORTED = -5  /* size outside the supported limits                 */
};

/* Working precision of the search contractions (right environments,
 * conditional marginals, beam-update vectors): FP64, FP32, or BF16 inputs with
 * FP32 accumulation.  The boundary MPS itself (its GEMMs and the QR/SVD
 * factorisations), energies and accumulated scores are always FP64. */
enum { SPG_FP64 = 0, SPG_FP32 = 1, SPG_BF16 = 2 };

typedef struct spg_peps spg_peps_t;
typedef struct spg_env spg_env_t;

/* A Potts instance, Eq. (1): E(x) = sum_edges E_mn(x_m, x_n) + sum_sites E_n(x_n).
 * All pointers are HOST float64 arrays, row-major, read only during
 * spg_build_peps.  Edge classes: H (r,c)-(r,c+1), V (r,c)-(r+1,c),
 * D (r,c)-(r+1,c+1), A (r,c+1)-(r+1,c); a pair table is indexed
 * [state of the first site][state of the second site]. */
typedef struct {
  int32_t rows, cols, d;
  int32_t kings;              /* 1: H, V, D and A edges (king's graph); 0: H and V only */
  double beta;                /* inverse temperature of the Boltzmann weights exp(-beta E) */
  const double *local_E;      /* [rows][cols][d]                                        */
  const double *pair_E_h;     /* [rows][cols-1][d][d]                                   */
  const double *pair_E_v;     /* [rows-1][cols][d][d]                                   */
  const double *pair_E_d;     /* [rows-1][cols-1][d][d]; NULL when kings == 0           */
  const double *pair_E_a;     /* [rows-1][cols-1][d][d]; NULL when kings == 0           */
} spg_instance_desc;

/* Boundary-MPS contraction parameters (the paper's MpsParameters: bond
 * dimension and number of sweeps; "SVDTruncate" is the truncated SVD of
 * two-site blocks by randomized subspace iteration). */
typedef struct {
  int32_t chi;          /* bond dimension cap of every boundary MPS                 */
  int32_t num_sweeps;   /* variational sweeps per row (>= 1); one sweep is a       */
                        /* left-to-right then a right-to-left pass                  */
  int32_t precision;    /* SPG_FP64 / SPG_FP32 / SPG_BF16: search contractions      */
  int32_t oversample;   /* sketch oversampling p of the truncated SVD (>= 0)       */
  int32_t power_iters;  /* subspace (power) iterations q of the truncated SVD      */
} spg_mps_params;

/* Search parameters (the paper's SearchParameters). */
typedef struct spg_proposal spg_proposal_t;
typedef struct {
  int32_t max_states;   /* beam width M: partial configurations kept per step      */
  double cut_off_prob;  /* 0 disables; else a child whose probability is below     */
                        /* cut_off_prob times the best child of the step is        */
                        /* discarded (kept only as -inf padding)                   */
  const spg_proposal_t *proposal;  /* NULL: every child evaluated exactly; else    */
                        /* the learned proposal ranks children first (see below)   */
  double kappa;         /* with a proposal: about kappa * max_states children are  */
                        /* evaluated exactly per step before the guard (> 0)       */
  int32_t merge_branches;  /* != 0: children of a step whose frontiers (states of  */
                        /* the last cols + 1 sites, own state included) are equal */
                        /* are merged: only the one with the lowest energy of its  */
                        /* fixed sites (ties: lowest b*d + s) keeps its score      */
                        /* (Sec. 3.1 merge of branches); not with a proposal       */
  double droplet_energy;   /* with max_droplets > 0: largest energy gap of a      */
                        /* droplet above its state (>= 0)                          */
  int32_t droplet_hamming; /* a droplet must differ from its state and from each  */
                        /* droplet the state holds in more than this many sites   */
  int32_t max_droplets;    /* 0: none; else up to this many (<= SPG_MAX_DROPLETS) */
                        /* low-energy excitations kept per state while merging     */
                        /* branches (Sec. 3.1 low-energy excitations): the member */
                        /* of a merged group next after the kept one in (energy,  */
                        /* id) order differs from it only in sites no later site  */
                        /* couples to, so its energy gap is final; a state        */
                        /* inherits its parent's droplets and takes its group's   */
                        /* runner-up if the gap and Hamming tests pass. Needs     */
                        /* merge_branches; read them with spg_droplets            */
} spg_search_params;

#define SPG_MAX_DROPLETS 64

/* Build the PEPS of an instance (Sec. 2, Fig. 1(c)): copies the energy tables
 * to the device and forms the Boltzmann weights w = exp(-beta (E - eps)) of
 * every table, eps = the table minimum (the shift only rescales Z).
 * Errors: SPG_ERR_INVALID (null desc/out/table), SPG_ERR_UNSUPPORTED (sizes),
 * SPG_ERR_NONFINITE (non-finite beta or energy), SPG_ERR_OOM, SPG_ERR_HIP.
 * Blocks until the tables are on the device. */
int spg_build_peps(const spg_instance_desc *desc, void *stream, spg_peps_t **out);

/* Boundary-MPS contraction of the PEPS (Sec. 2, Fig. 1(d); Sec. 2.1 names the
 * boundary-MPS approach): for r = rows-1 .. 0 the row's transfer operator is
 * applied to the previous boundary MPS and compressed to bond dimension chi.
 * The result (rows x cols tensors of chi_c x d x chi_{c+1}, plus per-row
 * log-scales) is held in a new env.  The bottom row is its exact chain of
 * nearest-neighbour factors at bond d (chi >= d); every other row has a unit-norm
 * centre at column 0, or at column 1 when column 0 kept its natural basis (at
 * most chi states, no rotation), with right isometries beyond it.  The call
 * returns when the stream has finished the contraction; when log_Z_out (HOST)
 * is not NULL it also writes the estimate of log Z.
 * Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED (chi, precision), SPG_ERR_OOM,
 * SPG_ERR_HIP, SPG_ERR_NONFINITE (log Z requested and not finite). */
int spg_boundary_mps(const spg_peps_t *peps, const spg_mps_params *params, void *stream,
                     spg_env_t **out, double *log_Z_out);

/* Conditional marginals (Sec. 2: marginal and conditional probabilities are
 * derived from the contraction): for each of n_beam partial configurations
 * b (DEVICE int32 [n_beam][rows*cols], entries of sites < `site` used),
 * writes log p(x_site = s | b) for s = 0..d-1 to log_cond_out (DEVICE float64
 * [n_beam][d]).  Impossible states get -inf.
 * Errors: SPG_ERR_INVALID (null pointers, site out of range, n_beam < 1),
 * SPG_ERR_OOM, SPG_ERR_HIP. */
int spg_marginals(const spg_env_t *env, int32_t site, int32_t n_beam, const int32_t *beam_cfg,
                  double *log_cond_out, void *stream);

/* spg_marginals for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * Same arguments and the same results (same kernels, bitwise), but every work
 * buffer lies in one static 64 MiB device array per GPU, which the library
 * holds until the process ends; the call allocates nothing.  A call needs
 *   FP64 env:     256-byte-rounded parts n_beam*rows*cols + 4 n_beam
 *                 + 8 n_beam (cols+1) chi + 8 n_beam chi  bytes,
 *   FP32/BF16:    n_beam*rows*cols + 4 n_beam + 4 n_beam (cols+1) chi
 *                 + 4 n_beam chi + 8 n_beam chi + 4 n_beam chi d  bytes,
 * at most 64 MiB (n_beam = 4096 fits at rows = cols = 12, chi = 64); a larger
 * call returns SPG_ERR_INVALID before any launch.  Every call on one GPU uses
 * the same array, which keeps the last call's contents and is cleared by each
 * call (a fill kernel on `stream`): calls that overlap on one GPU (two streams
 * or threads) race and must be serialised by the caller.  The env's device
 * must be the current device.
 * Errors: as spg_marginals; SPG_ERR_INVALID (scratch too small, wrong current
 * device); SPG_ERR_HIP (the scratch's address cannot be obtained). */
int spg_marginals_noalloc(const spg_env_t *env, int32_t site, int32_t n_beam,
                          const int32_t *beam_cfg, double *log_cond_out, void *stream);

/* Branch-and-bound search (Sec. 2; Fig. 1(d)-(e)): visits the sites in
 * row-major order, keeping the max_states most probable partial
 * configurations (ties: parent position, then state), and returns the final
 * beam: the states with a finite log-probability first, sorted by energy
 * ascending (ties: beam position), then the beam's other slots.
 * With params->proposal set, each step first ranks the children with the
 * network, evaluates exactly only the best-ranked ones (about kappa *
 * max_states), and bounds every other child of parent b by b's unevaluated
 * weight Z_b - sum of its evaluated q (plus a relative floor: 1e-9 of Z_b on
 * FP64 envs, 1e-3 on FP32 and 3e-2 on BF16 ones, where Z_b is known to that
 * precision), where Z_b = L^b R_c comes from the right environments at no
 * extra cost; parents whose bound reaches a lower bound of the
 * max_states-th exact score are evaluated in full.  The finite part of the
 * result is then the plain search's whatever the network predicts (exact up
 * to the floor while no conditional weight is negative, i.e. outside the
 * truncation-error regime).  Outputs:
 *   states_out   DEVICE int32   [max_states][rows*cols]
 *   energies_out DEVICE float64 [max_states]  (Eq. (1), recomputed in FP64)
 *   logp_out     DEVICE float64 [max_states]  (accumulated log-probability)
 *   n_out        HOST   int32   number of rows written with a finite log-probability
 *                                (rows beyond the beam size are left untouched)
 * Synchronises the stream (n_out is a host output).
 * Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED (max_states), SPG_ERR_OOM, SPG_ERR_HIP. */
int spg_branch_and_bound(const spg_env_t *env, const spg_search_params *params,
                         int32_t *states_out, double *energies_out, double *logp_out,
                         int32_t *n_out, void *stream);

/* The pruning step of the branch-and-bound search (Sec. 2: a fixed number of
 * the most probable configurations is kept at every variable): the indices of
 * the min(M, n) largest of n scores, ordered by score descending and, among
 * equal scores, by index ascending; NaN ranks as -inf.
 *   scores      DEVICE float64 [n]
 *   sel_out     DEVICE int32   [min(M, n)]
 *   scores_out  DEVICE float64 [min(M, n)] the selected scores, or NULL
 * The same selection spg_branch_and_bound applies to each step's d*beam
 * candidates.  Allocates its work buffers per call (device-synchronous).
 * Errors: SPG_ERR_INVALID (n < 0, M < 1, null scores/sel_out with n > 0),
 * SPG_ERR_OOM, SPG_ERR_HIP. */
int spg_topm(int32_t n, int32_t M, const double *scores, int32_t *sel_out, double *scores_out,
             void *stream);

void spg_free_peps(spg_peps_t *peps);
void spg_free_env(spg_env_t *env);
const char *spg_last_error(void);

/* ---- batches ------------------------------------------------------------
 * Many independent instances (each its own lattice size, d, chi and beam)
 * run as one unit: every instance's contraction and search is enqueued on
 * one of n_streams streams (round-robin; instances sharing a stream share one
 * contraction workspace), forked from and joined back into the caller's
 * stream.  With use_graph the whole batch is captured once into a HIP graph
 * and later runs replay it as a single launch.  Each instance's results are
 * those of spg_boundary_mps + spg_branch_and_bound on it with the same GEMM
 * tile (bitwise: the kernels are deterministic). */
typedef struct spg_batch spg_batch_t;
typedef struct {
  int32_t chi, num_sweeps, precision, oversample, power_iters;  /* as spg_mps_params */
  int32_t max_states;                                           /* as spg_search_params */
  double cut_off_prob;
} spg_batch_item;

/* flags: SPG_BATCH_CLASSES groups FP64 instances of equal shape (rows,
 * cols, d, lattice kind, chi, beam, sweeps, truncation parameters, cut-off)
 * into classes whose members share every launch: each kernel of the path runs
 * once per class with one workgroup set per member.  Other instances run one
 * by one on the streams. */
#define SPG_BATCH_CLASSES 1

/* peps HOST array [n] of PEPS handles (the batch copies their tables; they
 * must stay alive while the batch exists), items HOST [n].  Allocates every
 * per-instance buffer.  Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED,
 * SPG_ERR_OOM, SPG_ERR_HIP. */
int spg_batch_create(const spg_peps_t *const *peps, const spg_batch_item *items, int32_t n,
                     int32_t n_streams, int32_t flags, spg_batch_t **out);
/* Number of units (classes and single instances) and, in unit_of HOST int32
 * [n] (may be NULL), the unit of each instance. */
int spg_batch_info(const spg_batch_t *batch, int32_t *n_units, int32_t *unit_of);
/* The plan spg_batch_create would make for instances of these shapes, on the
 * host only (no device call, nothing allocated; a batch of many instances of
 * the method, Sec. 3.1, checked before it is built).  shapes HOST int32
 * [n][4] = (rows, cols, d, kings) of each instance; items, n, flags as for
 * spg_batch_create.  Outputs, all HOST: unit_of int32 [n], the unit of each
 * instance; n_units; unit_bytes int64 [n][2] = (members, slice bytes) of each
 * unit u < n_units (slice 0 for a single instance, whose buffers are its own
 * allocations); n_buffers int32 [n], the buffers of each class's slice;
 * layout int64 [n][max_buffers][2] (NULL when max_buffers = 0) = (offset,
 * bytes) of each buffer in the slice, filled for classes of at most
 * max_buffers buffers.  A class allocates members x slice bytes, members at
 * a stride of one slice.  Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED. */
int spg_batch_plan(const int32_t *shapes, const spg_batch_item *items, int32_t n, int32_t flags,
                   int32_t *unit_of, int32_t *n_units, int64_t *unit_bytes, int32_t max_buffers,
                   int64_t *layout, int32_t *n_buffers);
void spg_batch_free(spg_batch_t *batch);
/* Runs every instance (asynchronous on `stream`).  The first run is eager
 * and synchronises once (it sizes the workspaces); with use_graph != 0 the
 * following runs capture the batch into a graph (once) and replay it. */
int spg_batch_run(spg_batch_t *batch, int32_t use_graph, void *stream);
/* Results of instance i after a run (synchronises the device): n_out HOST =
 * rows with finite log-probability; the first n_out rows of its states
 * (int32 [.][rows*cols]), energies and log-probabilities (float64, sorted by
 * energy) are copied to the caller's DEVICE buffers states_out, energies_out,
 * logp_out (each may be NULL); log_Z HOST (may be NULL) = its log Z. */
int spg_batch_result(const spg_batch_t *batch, int32_t i, int32_t *states_out,
                     double *energies_out, double *logp_out, int32_t *n_out, double *log_Z);
/* GEMM output tile (32 or 64) of instance i's unit; drops a captured graph. */
int spg_batch_set_tuning(spg_batch_t *batch, int32_t i, int32_t gemm_tile);
/* Autotuner: times every unit (class or single instance) and, one knob after
 * the other, keeps the fastest GEMM tile (64 or 32), then the faster form of
 * the MPO d-index contractions and of the Q formation of one-panel QRs (the
 * two forms of each give bitwise equal results, see spg_set_kernel_forms);
 * reruns the batch with the choices (synchronous).  tile_out HOST int32 [n]
 * (may be NULL): the tile of each instance. */
int spg_batch_autotune(spg_batch_t *batch, void *stream, int32_t *tile_out);
/* The launch choices of instance i's unit, each output HOST and optional: the
 * GEMM tile, the MPO contraction form and the Q formation (1 = the column /
 * split forms, as in spg_set_kernel_forms).  SPG_ERR_INVALID for a bad index. */
int spg_batch_tuning(const spg_batch_t *batch, int32_t i, int32_t *gemm_tile,
                     int32_t *mpo_columns, int32_t *q_split);
/* Process default GEMM tile (32 or 64) of calls outside batches on this thread. */
int spg_set_tuning(int32_t gemm_tile);
/* Process defaults, on this thread, of two kernel forms of the boundary MPS
 * (Sec. 2: the row transfer operator applied to the boundary MPS, then
 * truncated); each pair of forms gives bitwise equal results.  Batches created
 * afterwards keep the setting.  mpo_columns, the MPO's d-index contractions:
 * 1 (default) for d in {8, 16, 24, 32} one thread per source column computes
 * the d outputs that share it, each source entry read once; 0 one thread per
 * output (other d up to 32 always take it; above d = 32 these contractions
 * are batched GEMMs on the matrix cores whatever the setting).  q_split, the
 * orthonormal factor Q of the truncation's QR factorisations of one panel (at
 * most 512 rows, 32 to 80 columns): 1 (default) the panel kernel stores its reflectors and a second
 * kernel forms Q with one compute unit per column; 0 the panel kernel forms Q
 * itself.  SPG_ERR_INVALID for values other than 0 and 1. */
int spg_set_kernel_forms(int32_t mpo_columns, int32_t q_split);
/* Reduced-precision form of the FP64 GEMMs (the precision form of the
 * boundary MPS's contractions with the MPO and its environments, Sec. 2; not
 * the default): with fp32_products = 1 every FP64 GEMM of calls on this thread
 * rounds its FP64 operands to FP32 and multiplies and accumulates in FP32 on
 * the matrix cores (v_mfma_f32_16x16x4f32), storing FP64 results; the QR, the
 * Jacobi SVD, the MPO d-index contractions and every normalisation stay FP64.
 * It covers the FP64 search's per-ancestor products as well, so set it around
 * the calls it is meant for.  0 (default) restores FP64 products.
 * SPG_ERR_INVALID for other values. */
int spg_set_gemm_precision(int32_t fp32_products);

/* ---- learned proposal ---------------------------------------------------
 * Not part of the paper's method: a 2-layer FP32 network that ranks the
 * children (b, s) of the beam so the exact contraction runs for few of them.
 * Per child, F = 6 features (each clamped at -30 and divided by 10 where the
 * value is a log-weight relative to its maximum): -beta dE(b, s) (Eq. (1)
 * terms closing at the site) relative to the best s; the one-step look-ahead
 * sum over the unexplored neighbours n of log sum_y exp(-beta (E_n(y) +
 * E_pair(s, y))) relative to the best s; log of the site's unconditioned
 * one-site weight of the boundary MPS relative to the best s; c / (cols - 1);
 * r / (rows - 1); score(b) minus the best score of the beam.
 * Network: h = relu(W1 f + b1) (H hidden units, 1 <= H <= 64),
 * logit = w2 . h + b2, p(s | b) = softmax over s.  Parameters (float32,
 * n = 8 H + 1): [W1 (H x F, row-major), b1 (H), w2 (H), b2].
 * Loss: cross-entropy against the exact conditionals, averaged over parents. */
#define SPG_PROPOSAL_FEATURES 6

typedef struct {
  int32_t epochs;        /* passes over the collected steps (>= 1)                 */
  float learning_rate;   /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8)      */
  int32_t max_states;    /* beam width of the exact search that provides targets  */
} spg_train_params;

/* New network with deterministic initial weights drawn from `seed`
 * (SplitMix64, uniform in +-sqrt(6 / fan_in), biases 0).  Owned by the caller,
 * released with spg_proposal_free.  Errors: SPG_ERR_INVALID, SPG_ERR_OOM. */
int spg_proposal_create(int32_t hidden, uint64_t seed, spg_proposal_t **out);
void spg_proposal_free(spg_proposal_t *prop);

/* Copy parameters out (host_out, HOST float32 [n], may be NULL) and/or in
 * (host_in, may be NULL; resets the Adam state); *n_params (HOST) receives n.
 * Synchronous. */
int spg_proposal_params(spg_proposal_t *prop, float *host_out, const float *host_in,
                        int32_t *n_params);

/* Train on one instance: runs the exact search of `env` with
 * tp->max_states, records every step's features and exact conditionals, then
 * takes tp->epochs passes over the steps in order, one Adam step per step.
 * Repeated calls continue the same optimiser state.  loss_out (HOST float32
 * [epochs], may be NULL) receives the mean loss of each pass.  Synchronises.
 * Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED (non-FP64 env), SPG_ERR_OOM,
 * SPG_ERR_HIP. */
int spg_proposal_train(spg_proposal_t *prop, const spg_env_t *env, const spg_train_params *tp,
                       void *stream, float *loss_out);

/* Building blocks of the training (tests, custom loops); all asynchronous.
 * Features of the children of n_beam partial configurations at `site`:
 * beam_cfg DEVICE int32 [n_beam][rows*cols], beam_score DEVICE float64
 * [n_beam] -> feats_out DEVICE float32 [n_beam][d][F]. */
int spg_proposal_features(const spg_env_t *env, int32_t site, int32_t n_beam,
                          const int32_t *beam_cfg, const double *beam_score, float *feats_out,
                          void *stream);
/* log p(s | b) of the network: feats DEVICE float32 [n_beam][d][F] ->
 * logp_out DEVICE float32 [n_beam][d]. */
int spg_proposal_forward(const spg_proposal_t *prop, int32_t n_beam, int32_t d,
                         const float *feats, float *logp_out, void *stream);
/* Loss and its gradient for targets target_logp DEVICE float32 [n_beam][d]
 * (-inf allowed): grad_out DEVICE float32 [n], loss_out DEVICE float32 [1].
 * Reduction order is fixed, so results are bitwise reproducible. */
int spg_proposal_loss_grad(const spg_proposal_t *prop, int32_t n_beam, int32_t d,
                           const float *feats, const float *target_logp, float *grad_out,
                           float *loss_out, void *stream);
/* One Adam step with gradient grad DEVICE float32 [n]. */
int spg_proposal_adam(spg_proposal_t *prop, const float *grad, float learning_rate,
                      void *stream);

/* Counters of the env's last spg_branch_and_bound call: counts[0] children
 * evaluated exactly (fallback evaluations included), counts[1] children
 * resolved (sum over steps of parents x d), counts[2] parents that fell back
 * to full evaluation.  HOST int64 [3].  Synchronous. */
/* Droplets of the state returned at position `state` (0-based, energy order)
 * by the last spg_branch_and_bound on this env, which must have run with
 * max_droplets > 0 (Sec. 3.1 low-energy excitations; the rule is described
 * with spg_search_params).  Writes min(count, max_out) whole configurations to
 * configs_out (HOST int32 [max_out][rows*cols], row-major sites) with their
 * Eq. (1) energies (the state's energy plus the recorded gap) to energies_out
 * (HOST [max_out]), in the order they were taken; *n_out = count.  Buffers are
 * caller-owned.  Blocks until the device is idle.
 * Errors: SPG_ERR_INVALID (null pointers, no droplets collected, state out of
 * range), SPG_ERR_HIP. */
int spg_droplets(const spg_env_t *env, int32_t state, int32_t max_out, int32_t *configs_out,
                 double *energies_out, int32_t *n_out);

/* Ising instance -> Potts tables of a lattice of spin clusters (host only, no
 * device work): the paper's Ising input (Sec. 2, Eq. (2)) grouped into the
 * Potts variables of Eq. (1) by a cluster assignment rule (Sec. 3.1).
 * E(s) = sum_q J_q s_{i_q} s_{j_q} over the n_terms listed terms (0-based
 * spin indices; i_q == j_q is a field J_q s_i; repeated terms add), s = +-1.
 * cluster_of[i] = r * cols + c places spin i (of n_spins = rows * cols * t) in
 * cluster (r, c); every cluster holds t spins (1 <= t <= 8), ordered by spin
 * index: the k-th is bit k of the cluster's state x, s = 2 bit_k(x) - 1, so
 * d = 2^t.  Couplings must join spins of one cluster or of neighbouring
 * clusters (r,c)-(r,c+1), (r,c)-(r+1,c), and with kings != 0 also
 * (r,c)-(r+1,c+1) and (r,c+1)-(r+1,c).  Writes the tables of
 * spg_instance_desc, in its layouts, to caller-owned HOST arrays: local_E
 * [rows*cols][d], pair_E_h [rows][cols-1][d][d], pair_E_v [rows-1][cols][d][d],
 * pair_E_d and pair_E_a [rows-1][cols-1][d][d] (these two only with kings;
 * tables of an absent edge class may be NULL).
 * Errors: SPG_ERR_INVALID (sizes, null pointers, indices out of range, a
 * cluster with more or fewer than t spins, a coupling between clusters that
 * are not neighbours), SPG_ERR_UNSUPPORTED (t outside 1..8), SPG_ERR_NONFINITE. */
int spg_ising_to_potts(int32_t n_spins, int32_t n_terms, const int32_t *term_i,
                       const int32_t *term_j, const double *term_J, int32_t rows, int32_t cols,
                       int32_t t, int32_t kings, const int32_t *cluster_of, double *local_E,
                       double *pair_E_h, double *pair_E_v, double *pair_E_d, double *pair_E_a);

int spg_search_stats(const spg_env_t *env, int64_t *counts);

/* ---- inspection hooks (tests and tools) -------------------------------- */

/* Sizes of an env: rows, cols, d, chi and the bond dimensions
 * bond_dims HOST int32 [rows][cols+1] (may be NULL).  Synchronous. */
int spg_env_info(const spg_env_t *env, int32_t *rows, int32_t *cols, int32_t *d, int32_t *chi,
                 int32_t *bond_dims);

/* Copy the boundary MPS to the host: tensors HOST float64
 * [rows][cols][chi][d][chi] (zero outside the bond dimensions) and
 * lam HOST float64 [rows] (log-scales; either may be NULL).  Synchronous. */
int spg_env_export(const spg_env_t *env, double *tensors, double *lam);

/* Make an env from given boundary-MPS tensors (HOST float64, same layout as
 * spg_env_export, bond dimensions HOST int32 [rows][cols+1]) so the search
 * can be run on tensors computed elsewhere.  `precision` selects the search
 * arithmetic as in spg_mps_params.  Errors: SPG_ERR_INVALID, SPG_ERR_UNSUPPORTED,
 * SPG_ERR_OOM, SPG_ERR_HIP.  Blocks until the copy is done. */
int spg_env_import(const spg_peps_t *peps, int32_t chi, const int32_t *bond_dims,
                   const double *tensors, const double *lam, int32_t precision, void *stream,
                   spg_env_t **out);

/* Opt-in kernel timing: while enabled, every launch of a timed kernel class
 * ("gemm_f64", "qr_f64", "jacobi_svd_f64", "normalize_box", "right_env",
 * "marginals", "select_topm", "beam_update", "final_sort", "propose",
 * "guided_eval", "mlp_grad", "merge_branches") is bracketed by HIP
 * events recorded on the stream it is launched on.  spg_profile_query
 * synchronises on those events and returns, since the last reset, the number
 * of launches, their summed duration in milliseconds and (total_work, may be
 * NULL) their summed algorithmic work: flops for the contraction classes
 * (gemm_f64, qr_f64, right_env, marginals, beam_update), bytes for
 * normalize_box and select_topm, 0 for the others.  Not thread-safe. */
void spg_profile_enable(int32_t on);
void spg_profile_reset(void);
int spg_profile_query(const char *name, int64_t *count, double *total_ms, double *total_work);

#ifdef __cplusplus
}
#endif
#endif /* SPG_H */
