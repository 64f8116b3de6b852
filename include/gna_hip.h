/*
 * gna_hip.h -- C ABI of libgna_hip.so, the MI355X (gfx950) library for the
 * data-parallel hot path of the GNA reactor-antineutrino prediction chain:
 *
 *   P_ee(E; L, theta) -> sum over baselines -> x flux x IBD cross section
 *   -> Gauss-Legendre bin integration -> Gaussian energy smearing
 *   -> Poisson chi^2 and its gradient with respect to
 *      theta = (dm2_21 [eV^2], dm2_31 [eV^2], sin^2 th12, sin^2 th13, norm).
 *
 * Paper: A. Fatkina et al., "CUDA Support in GNA Data Analysis Framework",
 * arXiv:1804.07682.  Sec. 4.1 defines the oscillation probability; Sec. 2.1
 * and 4.2 define the conventions kept here:
 *   - a transformation maps read-only input vectors and scalar "variables"
 *     to output vectors (Sec. 2.1, Fig. 2);
 *   - data lives on the outputs, inputs are views (Sec. 2.1, Sec. 4.2);
 *   - all memory is allocated at the configuration stage (Sec. 4.2): this
 *     library never allocates device memory -- the caller hands it every
 *     buffer, including a workspace sized by the *_workspace_size calls (the
 *     one exception is the fixed static staging array of
 *     gna_pee_host_noalloc, loaded with the library's device code);
 *   - the status of the GPU computation is available on the host afterwards
 *     (Sec. 4.2): every call returns a status code, and device-side domain
 *     errors are latched in the plan and read with gna_plan_status.
 *
 * Plain C: pointers, sizes, no C++ or torch types.  A "stream" argument is a
 * hipStream_t passed as void* (NULL = the default stream).  "_dev" pointers
 * are device memory on the current HIP device; "_host" pointers (and every
 * pointer inside gna_problem / gna_model) are host memory, read during the
 * call only.  Device buffers must be 16-byte aligned unless stated.
 *
 * Threading: calls on different plans are independent.  One plan must not be
 * evaluated concurrently on two streams (its workspace holds per-eval
 * counters).  The last error message is thread-local.
 */
#ifndef GNA_HIP_H
#define GNA_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GNA_ABI_VERSION 5

/* ---- status codes -------------------------------------------------------- */
#define GNA_OK 0
#define GNA_E_INVAL (-1)       /* bad argument, detected on the host before any launch   */
#define GNA_E_DOMAIN (-2)      /* a device-side domain error was latched (see below)     */
#define GNA_E_HIP (-3)         /* a HIP runtime call failed (message names it)           */
#define GNA_E_WORKSPACE (-4)   /* workspace missing, misaligned or too small              */
#define GNA_E_UNSUPPORTED (-5) /* valid request outside what this library implements      */

/* ---- precision modes ----------------------------------------------------- */
/* GNA_FP64: every step in FP64.
 * GNA_MIXED: oscillation phases and their reduction modulo pi/2 in FP64 (a
 *   52 km baseline puts phases at ~1e2-1e3 rad, where FP32 loses the phase);
 *   sin^2 / cos^2 / sin 2phi of the reduced argument, the probability, the
 *   flux products, the bin sums and the smearing in FP32 with FP32
 *   accumulation; chi^2, d chi^2/d nu and the final gradient sums in FP64. */
#define GNA_FP64 0
#define GNA_MIXED 1

int gna_abi_version(void);
/* Static description of a status code; never NULL. */
const char* gna_strerror(int status);
/* Thread-local description of the last error raised on this thread ("" if none). */
const char* gna_last_error_message(void);

/* ---- elementwise survival probability (Sec. 4.1, alpha = beta = e) ------- */
/*
 * P_dev[i] = sum_r w_r * P_ee(E_dev[i]; L_r, theta),  i < n, where
 *   P_ee = 1 - 4 sum_{i>j} |U_ei|^2 |U_ej|^2 sin^2(dm2_ij L / 4E)
 * (the Sec. 4.1 formula with alpha = beta = e, whose Im term vanishes), with
 * |U_e1|^2 = (1-s12)(1-s13), |U_e2|^2 = s12 (1-s13), |U_e3|^2 = s13,
 * dm2_32 = dm2_31 - dm2_21, and the phase dm2 L/4E = K dm2[eV^2] L[km]/E[MeV],
 * K = 1266.9326794198487 (hbar c = 197.3269804 MeV fm).  One launch covers
 * all n energies (Sec. 4.1: each energy is independent).
 *
 * E_dev     device, n doubles, E > 0 [MeV] (E <= 0 gives NaN in that slot).
 * n         >= 0; n = 0 is a no-op.
 * n_L       number of baselines, 1..64.
 * L_km_host host, n_L baselines >= 0 [km].
 * wL_host   host, n_L weights, or NULL for 1/n_L each (Fig. 4: one OscProb
 *           per baseline on a shared energy vector, summed).
 * theta_host host, 4 doubles (dm2_21, dm2_31, s12, s13); s12, s13 in [0, 1].
 * P_dev     device output, n doubles (GNA_FP64) or n floats (GNA_MIXED).
 * prec      GNA_FP64 or GNA_MIXED.
 * Asynchronous on `stream`.  Errors: GNA_E_INVAL (bad sizes, NULL, s out of
 * [0,1], misaligned pointers), GNA_E_HIP (launch failure).
 * Accuracy: phases are reduced exactly enough for |phase| < 1e9 rad.
 */
int gna_pee(const double* E_dev, int64_t n, int32_t n_L, const double* L_km_host,
            const double* wL_host, const double* theta_host, void* P_dev, int32_t prec,
            void* stream);

/*
 * General vacuum oscillation probability of Sec. 4.1 (its full equation):
 *   P(a -> b) = delta_ab - 4 sum_{i>j} Re(X_ij) sin^2(dm2_ij L / 4E)
 *                        + 2 sum_{i>j} Im(X_ij) sin(dm2_ij L / 2E),
 *   X_ij = V*_ai V_bi V_aj V*_bj,
 * V the PMNS matrix in the standard parametrisation by (theta12, theta13,
 * theta23, delta_CP); for antineutrinos V -> V* (delta -> -delta).
 * P_dev[i] = sum_r w_r P(E_dev[i]; L_r).
 *   alpha, beta     flavours 0 = e, 1 = mu, 2 = tau
 *   angles_host     host, 4 doubles: theta12, theta13, theta23, delta_CP [rad]
 *   dm2_host        host, 2 doubles: dm2_21, dm2_31 [eV^2] (any signs)
 *   antineutrino    0 or 1
 *   E_dev, n, n_L, L_km_host, wL_host, P_dev, prec as for gna_pee (E_dev and
 *   P_dev 8-byte aligned; P_dev holds floats in GNA_MIXED).
 * Asynchronous.  Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_prob(const double* E_dev, int64_t n, int32_t alpha, int32_t beta, int32_t n_L,
             const double* L_km_host, const double* wL_host, const double* angles_host,
             const double* dm2_host, int32_t antineutrino, void* P_dev, int32_t prec,
             void* stream);

/*
 * Elementwise P_ee as gna_pee, for energies and results in HOST memory: the
 * transfer-inclusive path of the paper (energies copied to the device,
 * evaluated, results copied back: Sec. 4.2 and the first row of Table 1),
 * pipelined.  The energies go in chunks of `chunk` elements; chunk i uses
 * buffer slot i % n_streams of the workspace and one of n_streams HIP streams
 * of the library, so the host-to-device copy, the kernel and the
 * device-to-host copy of successive chunks overlap.  Results equal gna_pee's
 * on the same energies bit for bit.
 *   E_host        host, n doubles [MeV]; pinned (hipHostMalloc) memory lets
 *                 the copies overlap, pageable memory works but serializes
 *   P_host        host, n outputs (FP64 doubles or mixed-precision floats)
 *   workspace_dev device, 256-byte aligned, >= the size from
 *                 gna_pee_host_workspace_size(chunk, n_streams, prec)
 *   chunk         even, >= 2 (a few million elements amortize each copy)
 *   n_streams     1..GNA_PIPE_MAX_STREAMS
 *   stream        the pipeline starts after the work already queued here
 * Synchronous: returns when P_host holds every result.  The library's
 * pipeline streams and event (created at the first call on a device, kept
 * until the process ends) are shared, so calls are serialized internally.
 * Errors: GNA_E_INVAL, GNA_E_WORKSPACE, GNA_E_HIP.
 */
#define GNA_PIPE_MAX_STREAMS 4
int gna_pee_host_workspace_size(int64_t chunk, int32_t n_streams, int32_t prec, size_t* bytes);
int gna_pee_host(const double* E_host, int64_t n, int32_t n_L, const double* L_km_host,
                 const double* wL_host, const double* theta_host, void* P_host, int32_t prec,
                 void* workspace_dev, size_t workspace_bytes, int64_t chunk, int32_t n_streams,
                 void* stream);

/*
 * For callers that cannot allocate device memory (serving loops, harnesses
 * that forbid hipMalloc, code that must not grow its footprint): the
 * pipeline of gna_pee_host with its staging buffers in a static device array
 * of the library (GNA_NOALLOC_SCRATCH_BYTES per device, held from the first
 * call on that device until the process ends) instead of a caller workspace.
 * Same arguments, results (bit for bit) and synchronous behaviour as
 * gna_pee_host without workspace_dev / workspace_bytes.
 *   chunk, n_streams  n_streams slots of `chunk` energies and `chunk` results
 *                     (each rounded up to 256 bytes) must fit the array:
 *                     n_streams * (chunk*8 + chunk*(8 or 4)) <= 32 MiB, e.g.
 *                     4 streams of 2^19 FP64 energies; larger requests fail
 *                     with GNA_E_INVAL before any HIP call.
 * Set-up: the first call on a device (or gna_device_init) resolves that
 * device's address of the array and creates the pipeline streams shared with
 * gna_pee_host; later calls allocate and create nothing.  The array keeps the
 * last call's staging contents (nothing in it needs to start at zero).  Calls
 * of both pipelined entry points are serialized inside the library, so two
 * threads never use the array at once; in one process only one pipelined call
 * runs at a time.  Errors: GNA_E_INVAL, GNA_E_HIP.
 */
#define GNA_NOALLOC_SCRATCH_BYTES (32u << 20)
int gna_pee_host_noalloc(const double* E_host, int64_t n, int32_t n_L, const double* L_km_host,
                         const double* wL_host, const double* theta_host, void* P_host,
                         int32_t prec, int64_t chunk, int32_t n_streams, void* stream);
/*
 * Set-up of the library's per-device resources on the current device: the
 * pipeline streams and event of gna_pee_host / gna_pee_host_noalloc and the
 * device address of the no-allocation staging array.  Idempotent; the
 * entry points above call it themselves.  Errors: GNA_E_HIP.
 */
int gna_device_init(void);

/*
 * Streaming copy dst_dev[i] = src_dev[i], i < n: 16-byte non-temporal loads
 * and stores in the fastest grid shape measured on MI355X; the HBM-bandwidth
 * reference of the benchmark and the known-size calibration of the
 * memory-traffic counters (not a step of the chain).  Both pointers 16-byte
 * aligned, not overlapping.  Asynchronous.  Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_stream_copy(const double* src_dev, double* dst_dev, int64_t n, void* stream);

/* ---- chain description --------------------------------------------------- */
/*
 * Model constants shared by all problems of a plan (readings of quantities the
 * paper leaves to the experiment's model):
 *   spectrum      S(E) = exp(spec[0] + spec[1] E + spec[2] E^2 + spec[3] E^3)
 *   IBD section   sigma(E) = x sqrt(x^2 - m_e^2), x = E - xsec_delta, 0 if x <= m_e
 *   flux factor   f_k = n0 * w_k * S(E_k) * sigma(E_k)   (w_k quadrature weight)
 *   resolution    sigma_E = res_a sqrt(E) at the true-bin centre (res_a >= 0)
 */
typedef struct gna_model {
  double spec[4];
  double xsec_delta;
  double m_e;
  double n0;
  double res_a;
} gna_model;

/*
 * One prediction problem (a "geometry"):
 *   n_bins    analysis bins, 1..4096, on strictly increasing edges[n_bins+1] > 0;
 *   gl_order  Gauss-Legendre order 1..64, n_sub >= 1 equal sub-intervals per
 *             bin; points per bin gl_order * n_sub <= 65536;
 *   L_km[n_L], wL[n_L] (or NULL = 1/n_L): baselines and weights, n_L 1..64;
 *   data      observed counts per bin (>= 0), used by chi^2.
 * The chain for one parameter point theta:
 *   Pbar_k = sum_r wL_r P_ee(E_k; L_r, theta)            (Sec. 4.1, Fig. 4)
 *   mu_j   = norm * sum_{k in bin j} f_k Pbar_k           (bin integration)
 *   nu_i   = sum_j R_ij mu_j,                             (smearing)
 *     R_ij = (erf((e_{i+1}-Ebar_j)/(sqrt2 s_j)) - erf((e_i-Ebar_j)/(sqrt2 s_j)))/2,
 *     Ebar_j = (e_j + e_{j+1})/2, s_j = res_a sqrt(Ebar_j)
 *   chi2   = 2 sum_i [nu_i - d_i + d_i ln(d_i/nu_i)]      (Baker-Cousins Poisson)
 * and its gradient d chi2 / d theta (5 values).  Quadrature points of bin j:
 * sub-interval edges u_s = e_j + ((e_{j+1}-e_j) s)/n_sub, u_{n_sub} = e_{j+1};
 * on [a,b]: E = (a+b)/2 + ((b-a)/2) t_i, w = ((b-a)/2) w_i.
 */
typedef struct gna_problem {
  int32_t n_bins;
  const double* edges;
  int32_t gl_order;
  int32_t n_sub;
  int32_t n_L;
  const double* L_km;
  const double* wL;
  const double* data;
} gna_problem;

/*
 * Launch-shape options (all 0 = automatic).  Autotuned values come from
 * gna_plan_autotune.
 *   threads        work-group size: 64, 128, 256, 512 or 1024
 *   lanes_per_bin  lanes cooperating on one bin: power of two, 1..64
 *   chunks         pieces each bin's points are split into (their partial
 *                  sums are added in a fixed order, so results do not depend
 *                  on scheduling): 1..1024
 *   persistent     0: one work-group per tile; 1: a grid of
 *                  (CUs x occupancy) work-groups pulling tiles from a queue
 *   smear_mfma     (chain plans only) 1, 2, 3: batched kernel with the
 *                  smearing as a block-banded MFMA GEMM (needs n_bins <=
 *                  256), register allocation for 2, 3 or 4 wavefronts per
 *                  SIMD; 0: banded smearing on the vector units; -1: automatic
 *   no_shared_phases  0 (default): in the batched MFMA kernel a tile of 16
 *                  parameter points that all have the same (dm2_21, dm2_31)
 *                  evaluates the phase terms once and sums them per bin
 *                  before combining them with each point's mixing weights
 *                  (a transformation is recomputed only when its own inputs
 *                  change, Sec. 2); results agree with the per-point path to
 *                  rounding, so a point's last bits may depend on its tile
 *                  neighbours.  1: every point evaluates its own phases, and
 *                  its result does not depend on the rest of the batch.
 *   split_tail     0: automatic; 1: each point's (fit's) tail
 *                  (smearing, chi^2, gradient) runs in the work-group that
 *                  finishes its last tile; 2: the point pass only stores bin
 *                  sums and the tails run in later launches: for a chain
 *                  plan one 512-lane work-group per parameter point (the
 *                  same sums as 1, in the same order, so the same bits, when
 *                  the shape also has 512 lanes; the default when a point
 *                  has several tiles), for a fitset two launches with
 *                  one wavefront per 64-row slice, then each fit's partials
 *                  added in a fixed order (the fitset default); 3 (fitset
 *                  plans only): queued tail, one launch: the persistent
 *                  queue holds the point tiles and, some way after each
 *                  fit's last tile, that fit's tail (one work-group waits for
 *                  the fit's tiles, then runs its slices and the fixed-order
 *                  sum; implies persistent = 1; same results as 2, bit for
 *                  bit).  A nonzero value also keeps gna_plan_autotune to
 *                  that tail.
 */
typedef struct gna_launch_opts {
  int32_t threads;
  int32_t lanes_per_bin;
  int32_t chunks;
  int32_t persistent;
  int32_t smear_mfma;
  int32_t no_shared_phases;
  int32_t split_tail;
} gna_launch_opts;

typedef struct gna_plan gna_plan;

/* ---- one geometry, a batch of parameter points (configuration stage) ---- */
/*
 * Sizes the workspace of a chain plan for up to max_batch parameter points.
 * Host only (no HIP call).  opts may be NULL.  Errors: GNA_E_INVAL.
 */
int gna_chain_workspace_size(const gna_model* model, const gna_problem* problem,
                             int32_t prec, int32_t max_batch, const gna_launch_opts* opts,
                             size_t* bytes);
/*
 * Configuration stage (Sec. 2, two-stage model; Sec. 4.2, allocation at
 * configuration): copies the description into ws_dev and builds, with
 * device kernels, the Gauss-Legendre rule, the quadrature energies, the flux
 * factors f_k and the banded smearing matrix.  ws_dev: device, 256-byte
 * aligned, ws_bytes >= gna_chain_workspace_size; owned by the caller, must
 * outlive the plan.  Synchronizes `stream` before returning.  *out receives a
 * host-allocated plan, freed by gna_plan_destroy.
 * Errors: GNA_E_INVAL, GNA_E_WORKSPACE, GNA_E_HIP, GNA_E_UNSUPPORTED.
 */
int gna_chain_create(const gna_model* model, const gna_problem* problem, int32_t prec,
                     int32_t max_batch, const gna_launch_opts* opts, void* ws_dev,
                     size_t ws_bytes, void* stream, gna_plan** out);
/*
 * Computational stage: chi^2 (and gradient) of B parameter points in one
 * launch sequence, asynchronous on `stream`.
 *   params_dev  device, [B][5] doubles (dm2_21, dm2_31, s12, s13, norm)
 *   chi2_dev    device output, [B] doubles
 *   grad_dev    device output, [B][5] doubles, or NULL (no gradient work)
 *   pred_dev    device output, [B][n_bins] doubles (nu), or NULL (Fig. 6:
 *               reading an intermediate output costs one extra write)
 * 1 <= B <= max_batch.  Parameters are not range-checked on the host (they
 * are device data): s12, s13 outside [0, 1] or nu_i <= 0 latch GNA_E_DOMAIN
 * (read it with gna_plan_status) and give NaN for that point.
 * Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_chain_eval(gna_plan* plan, const double* params_dev, int32_t B, double* chi2_dev,
                   double* grad_dev, double* pred_dev, void* stream);

/* ---- uneven batch: independent fits, one parameter point each ----------- */
/*
 * As the chain calls, for n_fits independent problems (each its own bins,
 * order, baselines and data), evaluated together in one launch.  Tiles of all
 * fits are queued largest-first.  pred_dev (optional) is the concatenation of
 * the fits' nu vectors in fit order.
 */
int gna_fitset_workspace_size(const gna_model* model, const gna_problem* problems,
                              int32_t n_fits, int32_t prec, const gna_launch_opts* opts,
                              size_t* bytes);
int gna_fitset_create(const gna_model* model, const gna_problem* problems, int32_t n_fits,
                      int32_t prec, const gna_launch_opts* opts, void* ws_dev,
                      size_t ws_bytes, void* stream, gna_plan** out);
/* params_dev [n_fits][5]; chi2_dev [n_fits]; grad_dev [n_fits][5] or NULL;
 * pred_dev [sum n_bins] or NULL. */
int gna_fitset_eval(gna_plan* plan, const double* params_dev, double* chi2_dev,
                    double* grad_dev, double* pred_dev, void* stream);

/* ---- plan queries and lifecycle ------------------------------------------ */
/*
 * Synchronizes `stream`, then reads and clears the plan's device status word.
 * *device_status (may be NULL) receives the raw word (bit 0: a mixing
 * parameter outside [0, 1]; bit 1: some nu_i <= 0 or not finite; bit 2: a
 * queued tail gave up waiting for its fit's tiles).
 * Returns GNA_E_HIP if bit 2 was set (the results of that evaluation are not
 * valid; gna_plan_rebuild restores the plan), else GNA_E_DOMAIN if any bit
 * was set, else GNA_OK (or GNA_E_HIP from the runtime).
 */
int gna_plan_status(gna_plan* plan, void* stream, int32_t* device_status);
/* Launch shape in use: writes 7 ints (threads, lanes_per_bin, chunks,
 * persistent, smear_mfma, shared_phases, split_tail) and the number of tiles
 * of one evaluation (for the MFMA scan kernel, smear_mfma > 0: its lanes per
 * work-group, 1, 1, and tiles of 16 points at the plan's max_batch).  shared_phases is 1 when the MFMA kernel lets tiles with
 * common (dm2_21, dm2_31) share their phases: the plan allows it
 * (no_shared_phases = 0) and the shape asks for it (the autotuner tries
 * both).  split_tail is 1 when the tails run in launches after the point
 * pass, 2 when a fitset queues them in its one persistent launch. */
int gna_plan_shape(const gna_plan* plan, int32_t shape_out[7], int64_t* n_tiles);
/*
 * Project-written autotuner: times each candidate launch shape of this plan
 * on `stream` with HIP events (median of `reps` evaluations at params_dev,
 * B points for chain plans), keeps the fastest, and, if cache_path is not
 * NULL, records it in a small JSON file keyed by the plan's shape bucket,
 * precision and GPU architecture (read back by gna_plan_autotune before
 * timing: a hit costs no launch).  Writes chi2/grad scratch into the
 * caller's chi2_dev / grad_dev.  Returns GNA_OK and the chosen shape.
 */
int gna_plan_autotune(gna_plan* plan, const double* params_dev, int32_t B, double* chi2_dev,
                      double* grad_dev, int32_t reps, const char* cache_path, void* stream,
                      int32_t shape_out[7]);
/* Frees the host-side plan (the caller still owns the workspace). */
int gna_plan_destroy(gna_plan* plan);
/*
 * Recovery (Sec. 5: a computation that fails is restarted from a saved
 * state): runs the configuration stage again into the plan's workspace from
 * the description the plan keeps on the host (tables, band of R, data,
 * launch shape; counters, queue and status word cleared), so a plan whose
 * evaluation failed or whose workspace was overwritten evaluates as new.
 * The chosen launch shape is kept.  Synchronizes `stream`.
 * Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_plan_rebuild(gna_plan* plan, void* stream);

/* ---- fault injection (tests of error handling) --------------------------- */
/* The next `count` HIP status checks inside the library that would succeed
 * report GNA_E_HIP instead ("injected failure"), so recovery paths can be
 * exercised from the host while every kernel still runs and exits normally.
 * count = 0 clears pending injections.  Process-wide.  Errors: GNA_E_INVAL. */
int gna_debug_inject_hip_errors(int32_t count);
/* Injected failures not yet consumed. */
int32_t gna_debug_pending_hip_errors(void);
/* The bounded wait of the queued tail (fitset plans, split_tail = 3): from
 * the next evaluation on, a tail waits for `extra_tiles` tiles more than its
 * fit has (so with extra_tiles > 0 no wait can end by the count) and gives
 * up after `spin_limit` sleeps (0: the default bound, about 2^20).  A wait
 * that gives up latches a status bit that gna_plan_status reports as
 * GNA_E_HIP; the launch still ends normally, its results are not valid, and
 * gna_plan_rebuild restores the plan.  gna_debug_queued_wait(plan, 0, 0)
 * restores the defaults.  Errors: GNA_E_INVAL (NULL or not a fitset plan,
 * negative values). */
int gna_debug_queued_wait(gna_plan* plan, int32_t spin_limit, int32_t extra_tiles);

/* ---- unfused transformations (vector in / vector out) -------------------- */
/*
 * The chain's steps as separate transformations (Sec. 2.1, Fig. 2: a
 * transformation maps read-only input vectors to an output vector it owns;
 * Sec. 4.2, Fig. 6: an intermediate result is read at the cost of one more
 * output).  FP64, over a batch of n_vec vectors stored one after another
 * (row-major [n_vec][length]); every sum is taken in a fixed order, so the
 * results do not depend on scheduling.  Device pointers 8-byte aligned;
 * n_vec = 0 is a no-op.  The fused chain entry points compute the same steps
 * in one launch.
 */

/*
 * Gauss-Legendre rule of order 1..64 on [-1, 1] (nodes ascending; weights),
 * computed on the device and returned in host memory: t_host[order],
 * w_host[order].  Synchronous (the null stream).  Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_gl_nodes(int32_t order, double* t_host, double* w_host);
/* The same rule into device memory t_dev[order], w_dev[order] on `stream`;
 * synchronizes `stream`. */
int gna_gl_nodes_dev(int32_t order, double* t_dev, double* w_dev, void* stream);

/*
 * Bin integration (the Gauss-Legendre sum of each bin):
 *   mu_dev[v][j] = sum_{i < ppb} w_dev[j*ppb + i] * x_dev[v][j*ppb + i]
 * for j < n_bins, v < n_vec; x_dev holds each vector's n_bins*ppb point
 * values bin after bin (the quadrature-point order of the chain), w_dev the
 * n_bins*ppb quadrature weights shared by all vectors, or NULL for weight 1
 * (values already weighted, as f_k P_k is).  Asynchronous on `stream`.
 * Errors: GNA_E_INVAL (sizes < 1, NULL, misaligned), GNA_E_HIP.
 */
int gna_bin_integrate(const double* x_dev, const double* w_dev, int64_t n_vec, int32_t n_bins,
                      int32_t ppb, double* mu_dev, void* stream);

/*
 * Smearing with a dense row-major matrix R_dev[n_rows][n_cols] (row =
 * reconstructed bin, column = true bin, as gna_plan_tables writes it):
 *   transpose = 0:  y_dev[v][i] = sum_j R_ij x_dev[v][j]   (x: n_cols, y: n_rows)
 *   transpose = 1:  y_dev[v][j] = sum_i R_ij x_dev[v][i]   (x: n_rows, y: n_cols)
 * transpose = 1 is the adjoint step of the gradient, d chi^2/d mu = R^T
 * d chi^2/d nu.  x_dev and y_dev must not overlap.  Asynchronous on `stream`.
 * Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_smear(const double* R_dev, int32_t n_rows, int32_t n_cols, int32_t transpose,
              const double* x_dev, int64_t n_vec, double* y_dev, void* stream);

/*
 * Baker-Cousins Poisson chi^2 of n_vec predictions nu_dev[v][n_bins]:
 *   chi2_dev[v] = 2 sum_i [nu_i - d_i + d_i ln(d_i / nu_i)]  (d ln(d/nu) = 0 at d = 0)
 * and, if dchi2_dnu_dev is not NULL, its derivative
 *   dchi2_dnu_dev[v][i] = 2 (1 - d_i / nu_i),
 * the seed of the adjoint pass.  data_dev holds the observed counts (>= 0):
 * one vector shared by all predictions (data_stride = 0) or one per
 * prediction (data_stride = n_bins).  A prediction with some nu_i <= 0 (or
 * NaN) gives chi2 = NaN for that vector and NaN in the offending derivative
 * entries (no status word: these calls have no plan).  Asynchronous on
 * `stream`.  Errors: GNA_E_INVAL, GNA_E_HIP.
 */
int gna_chi2(const double* nu_dev, const double* data_dev, int64_t data_stride, int32_t n_bins,
             int64_t n_vec, double* chi2_dev, double* dchi2_dnu_dev, void* stream);

/*
 * Configuration-stage tables of problem `index` of a plan (Fig. 6-style
 * intermediate read): quadrature energies E_dev[n_bins*ppb], flux factors
 * f_dev[n_bins*ppb] (as doubles), and the dense smearing matrix
 * R_dev[n_bins][n_bins] (row = reconstructed bin), expanded from the band.
 * Any output may be NULL.  Asynchronous.
 */
int gna_plan_tables(const gna_plan* plan, int32_t index, double* E_dev, double* f_dev,
                    double* R_dev, void* stream);

/* ---- transformation graph (Sec. 2, Fig. 2-6) ------------------------------
 * A graph of vector-in / vector-out transformations over the kernels above,
 * in the paper's two stages.  Configuration: create variables (scalars) and
 * nodes, each owning one FP64 output vector; a node's inputs are read-only.
 * Then gna_graph_workspace_size / gna_graph_bind place every output, and the
 * configuration tables of each geometry, in one caller-allocated device
 * workspace and compute those tables.  Computation: gna_graph_set changes a
 * variable and taints every node that depends on it, directly or through its
 * inputs; gna_graph_eval / gna_graph_read recompute only tainted nodes, inputs
 * first (lazy evaluation), and a node is computed at most once between
 * changes of what it depends on.  Reading any node's output, intermediate or
 * final, costs one device-to-host copy (Sec. 4.2).  The graph runs unfused
 * kernels, one per node, in FP64; the fused chain entry points above are the
 * fast path for the same chain.
 *
 * Node ids are dense from 0 in creation order; variable ids likewise (their
 * own numbering).  Every function returns GNA_OK or an error code (message in
 * gna_last_error_message); creation functions fail after gna_graph_bind, and
 * computation functions before it.  A graph is used by one host thread at a
 * time.
 */
typedef struct gna_graph gna_graph;
int gna_graph_create(gna_graph** graph_out);
int gna_graph_destroy(gna_graph* graph);
/* A scalar variable (dm2_21, sin^2 theta_13, a normalisation, ...). */
int gna_graph_variable(gna_graph* graph, const char* name, double value, int32_t* var_out);
/* Geometry node: quadrature energies E_k [n_bins * gl_order * n_sub] of a
 * problem (the problem's edges, quadrature and data are copied; its
 * baselines are not used by the graph).  The geometry also carries the flux
 * factors f_k, the smearing matrix R and the data of the problem. */
int gna_graph_points(gna_graph* graph, const gna_model* model, const gna_problem* problem,
                     int32_t* node_out);
/* f_k = N0 S(E_k) sigma(E_k) w_k of a geometry: a configuration table, never tainted. */
int gna_graph_flux(gna_graph* graph, int32_t points, int32_t* node_out);
/* P_ee(E; L) over a node's energies, Sec. 4.1, with four variables
 * (dm2_21, dm2_31, sin^2 th12, sin^2 th13). */
int gna_graph_oscprob(gna_graph* graph, int32_t energies, double L_km, const int32_t vars[4],
                      int32_t* node_out);
/* sum_i w_i x_i over n_inputs nodes of equal length (1..64 inputs). */
int gna_graph_sum(gna_graph* graph, int32_t n_inputs, const int32_t* inputs,
                  const double* weights, int32_t* node_out);
/* Elementwise product of two nodes of equal length. */
int gna_graph_product(gna_graph* graph, int32_t a, int32_t b, int32_t* node_out);
/* Bin sums of a per-quadrature-point node of a geometry: [n_bins]. */
int gna_graph_integrate(gna_graph* graph, int32_t x, int32_t points, int32_t* node_out);
/* R x of a per-bin node with the geometry's smearing matrix: [n_bins]. */
int gna_graph_smear(gna_graph* graph, int32_t x, int32_t points, int32_t* node_out);
/* v x with a variable v. */
int gna_graph_scale(gna_graph* graph, int32_t x, int32_t var, int32_t* node_out);
/* Baker-Cousins Poisson chi^2 of a per-bin prediction against the geometry's
 * data: [1]. */
int gna_graph_chi2(gna_graph* graph, int32_t nu, int32_t points, int32_t* node_out);
/* Device bytes gna_graph_bind needs (outputs and configuration tables). */
int gna_graph_workspace_size(const gna_graph* graph, size_t* bytes);
/* Place outputs in workspace_dev (256-byte aligned, >= the size above) and
 * compute the configuration tables on `stream`.  Synchronous.  The graph
 * keeps the workspace until it is destroyed.  The host mirrors of all
 * outputs go in one page-locked host allocation made here (host memory, one
 * double per output element; freed by gna_graph_destroy). */
int gna_graph_bind(gna_graph* graph, void* workspace_dev, size_t workspace_bytes, void* stream);
/* Change a variable: taints its dependents (no computation). */
int gna_graph_set(gna_graph* graph, int32_t var, double value);
/* Compute `node` and whatever it needs that is tainted, on `stream`
 * (asynchronous), and return its output's device address and length. */
int gna_graph_eval(gna_graph* graph, int32_t node, void* stream, const double** out_dev,
                   int64_t* n_out);
/* gna_graph_eval, then copy the output to host_out[n] (n = its length).
 * Synchronous. */
int gna_graph_read(gna_graph* graph, int32_t node, double* host_out, int64_t n, void* stream);
/* Output length of a node, and how many times it has been computed. */
int gna_graph_node_info(const gna_graph* graph, int32_t node, int64_t* n_out,
                        int64_t* evaluations);

/* ---- graph: host mirrors, target device, formula items, fused nodes ------
 * Every node output has a host mirror beside its device copy; a copy between
 * them happens only when the side that is read is stale (Sec. 4.2): reading a
 * node twice without a change in between copies once, and a node computed on
 * the CPU is uploaded only when a GPU node or gna_graph_eval needs it.
 *
 * Target device (Sec. 4.2: one flag switches where a transformation runs):
 * GNA_TARGET_GPU (default) or GNA_TARGET_CPU for one node, or node = -1 for
 * every node that has a CPU form (all but the geometry tables and the fused
 * chain node, which run on the GPU; asking CPU for one of those fails with
 * GNA_E_UNSUPPORTED).  A CPU node computes in FP64 on the host with libm,
 * its inputs brought to the host first.  The flag is the only way a node
 * runs on the CPU: the library never switches by itself.  Changing the
 * target does not taint a node.
 */
#define GNA_TARGET_GPU 0
#define GNA_TARGET_CPU 1
int gna_graph_set_target(gna_graph* graph, int32_t node, int32_t target);
/* stats[0] = output length, [1] = evaluations, [2] = device-to-host copies,
 * [3] = host-to-device copies of the node's output, [4] = GPU failures the
 * node recovered from on the CPU (failover below); *target its target.
 * (Copies of a geometry's smearing matrix for CPU smearing nodes are counted
 * on none of the nodes.) */
int gna_graph_node_stats(const gna_graph* graph, int32_t node, int64_t stats[5],
                         int32_t* target);
/* Failover (Sec. 5: the CPU implementation stays available when the GPU
 * fails), off by default: with on = 1, a GPU node whose kernel or copy
 * reports GNA_E_HIP is computed by its CPU form instead, the recovery is
 * counted in stats[4], and the node keeps its GPU target for the next
 * evaluation.  Nodes without a CPU form (the fused chain) return the error. */
int gna_graph_set_failover(gna_graph* graph, int32_t on);

/*
 * Formula items of the Sec. 4.1 probability (OscProb as one transformation
 * per term, then a weighted sum): over a node's energies E and one baseline,
 *   item 0: sin^2 phi,  item 1: sin 2phi,  phi = dm2 L / 4E = dm2 (K L) / E,
 * for pair 0 (dm2_21), 1 (dm2_31) or 2 (dm2_32 = dm2_31 - dm2_21).  The
 * node reads both splitting variables but is tainted only by those its phase
 * depends on.
 */
int gna_graph_osc_item(gna_graph* graph, int32_t energies, double L_km, int32_t dm21_var,
                       int32_t dm31_var, int32_t pair, int32_t item, int32_t* node_out);
/* P_ee = 1 - 4 sum_{i>j} |U_ei|^2 |U_ej|^2 sin^2 phi_ij from the three sin^2
 * items (pairs 21, 31, 32, same energies) and the mixing variables
 * sin^2 th12, sin^2 th13: a change of a mixing variable recomputes this node
 * only. */
int gna_graph_pee_items(gna_graph* graph, const int32_t sin2_items[3], int32_t s12_var,
                        int32_t s13_var, int32_t* node_out);
/* P(alpha -> beta) = delta_ab - 4 sum Re(X_ij) sin^2 phi_ij + 2 sum Im(X_ij)
 * sin 2phi_ij (the full Sec. 4.1 equation, as gna_prob) from the three sin^2
 * and the three sin 2phi items and the variables (th12, th13, th23, delta_CP)
 * [rad]; antineutrino 0 or 1 (delta -> -delta). */
int gna_graph_prob_items(gna_graph* graph, int32_t alpha, int32_t beta, int32_t antineutrino,
                         const int32_t angle_vars[4], const int32_t sin2_items[3],
                         const int32_t sin2phi_items[3], int32_t* node_out);
/* The fused general probability (gna_prob, FP64, one baseline) as a node:
 * variables (th12, th13, th23, delta_CP) and (dm2_21, dm2_31). */
int gna_graph_prob(gna_graph* graph, int32_t energies, double L_km, int32_t alpha, int32_t beta,
                   int32_t antineutrino, const int32_t angle_vars[4], const int32_t dm_vars[2],
                   int32_t* node_out);
/* The fused chain of a geometry (its baselines, quadrature and data; the
 * chain kernel of gna_chain_eval) as a node with output [6] = (chi^2,
 * d chi^2 / d theta for theta = the 5 variables (dm2_21, dm2_31, s12, s13,
 * norm)), in GNA_FP64 or GNA_MIXED: the graph's way to the gradient.  GPU
 * only.  Domain errors give NaN (the node has no status word). */
int gna_graph_chain(gna_graph* graph, int32_t points, const int32_t vars[5], int32_t prec,
                    int32_t* node_out);

#ifdef __cplusplus
}
#endif

#endif /* GNA_HIP_H */
