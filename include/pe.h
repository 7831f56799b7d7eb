/*
 * pe.h -- C ABI of the MI355X (gfx950) likelihood engine for metric-based
 * importance sampling of compact-binary gravitational-wave signals
 * (A. H. Nitz, "Robust, Rapid, and Simple Gravitational-wave Parameter
 * Estimation", arXiv:2410.05190).
 *
 * The library evaluates, for a large batch of proposal draws theta_i:
 *   - the noise-weighted inner product (a|b) = 4 Re int a* b / S_n df
 *     (Sec. II.A, Eq. 1), as a left-point sum over the half-open grid
 *     f_k = f_lo + k df, k = 0 .. n_bins-1;
 *   - the log-likelihood ratio against noise ln(L/L_n) = (d|h) - (h|h)/2
 *     (Sec. II.A, Eq. 3), either with an explicit coalescence phase or
 *     marginalised over a uniform one (ln I0(|Z|) - H/2);
 *   - the importance weights w_i = L_i pi_i / g_i (App. A.3, Eq. 5) and the
 *     effective sample size ESS = (sum w)^2 / sum w^2 (App. A.3, Eq. 6);
 *   - the waveform metric induced by the inner product (Sec. II.A), as the
 *     network Fisher matrix g_ij = sum_d (d_i h_d | d_j h_d) from central
 *     finite differences, and Gaussian proposal draws N(theta0, g^-1)
 *     (the local-metric proposal the paper names as its refinement, Sec. III.A).
 * The waveform is TaylorF2 (3.5PN phase, aligned spins, Newtonian amplitude)
 * cut at the test-mass ISCO of the total mass, projected onto long-wavelength
 * L-shaped detectors with light-travel delays.
 *
 * Conventions shared by every entry point:
 *   - Array arguments named *_dev are device pointers (HBM), owned by the
 *     caller; the library never frees them. Scalars are passed by value.
 *   - Every call enqueues work on `stream` (a hipStream_t; NULL = the null
 *     stream) and returns without synchronising, except pe_event_create and
 *     pe_event_status, which synchronise that stream.
 *   - Argument errors are detected on the host and returned at once; nothing
 *     is enqueued then. Errors found by kernels (bad PSD values, a metric that
 *     is not positive definite) are recorded in the event and returned by
 *     pe_event_status. A HIP error returns PE_ERR_HIP.
 *   - pe_last_error() gives a message for the last failing call of the
 *     calling thread.
 *   - An event handle is used by one host thread at a time. Results are
 *     bitwise reproducible for fixed inputs, precision and tile shape: no
 *     floating-point atomics are used.
 *
 * Parameters (units: solar masses, detector frame; Mpc; s; rad):
 *   PE_PARAMS_4D : theta = (Mc, eta, chi_eff, tc); one common real amplitude
 *                  amp0 on every detector, no delay. Always phase-marginalised.
 *   PE_PARAMS_11D: theta = (Mc, q, chi1z, chi2z, ra, dec, iota, psi, dL, tc,
 *                  phic), q = m2/m1 <= 1. ra, psi, phic are periodic
 *                  (2 pi, pi, 2 pi).
 * theta batches are structure-of-arrays: theta_dev[j*n + i] is parameter j of
 * draw i.
 */
#ifndef PE_H
#define PE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PE_MAX_DET 4
#define PE_MAX_DIM 11
#define PE_MAX_TM_POINTS 16384 /* tc nodes of a time-marginalised event */
#define PE_MIX_MAX 16          /* components of a mixture proposal (pe_mixture_logq) */

typedef struct pe_event_s *pe_event_t;

typedef enum {
    PE_OK = 0,
    PE_ERR_ARG = 1,       /* invalid argument, or invalid data/PSD values */
    PE_ERR_OOM = 2,       /* device allocation failed */
    PE_ERR_HIP = 3,       /* a HIP runtime call failed */
    PE_ERR_SINGULAR = 4,  /* the metric given to pe_draw is not positive definite */
    PE_ERR_NONFINITE = 5, /* data contains inf or nan */
    PE_ERR_BUDGET = 6,    /* request exceeds a fixed capacity */
    PE_ERR_TIMEOUT = 7    /* a wait ended before the request completed */
} pe_status_t;

/* PE_PREC_RELBIN: relative binning about the fiducial point of the last
 * pe_relbin_setup on the event (pe_loglike_batch only). */
typedef enum { PE_PREC_FP64 = 0, PE_PREC_SPLIT = 1, PE_PREC_RELBIN = 2 } pe_precision_t;
typedef enum { PE_PHASE_MARG = 0, PE_PHASE_EXPLICIT = 1 } pe_phase_t;
typedef enum { PE_PARAMS_4D = 0, PE_PARAMS_11D = 1 } pe_params_t;
/* Treatment of the luminosity distance (11-D only). PE_DIST_MARG: the
 * likelihood is marginalised over dL (Sec. III marginalises the extrinsic
 * parameters with analytic or numerical formulas; for the distance this is the
 * integral over the dL^2 prior of Singer & Price 2016), so theta's dL is
 * carried but never used: see pe_metric, pe_draw and pe_loglike_batch. */
typedef enum { PE_DIST_SAMPLED = 0, PE_DIST_MARG = 1 } pe_distance_t;
typedef enum { PE_C128 = 0, PE_C64 = 1 } pe_data_dtype_t;
typedef enum { PE_F64 = 0, PE_F32 = 1 } pe_psd_dtype_t;

/* Event description. det_geom[d] = {latitude, longitude, azimuth of the x arm
 * measured from north toward east}; the y arm is 90 degrees east of x. */
typedef struct {
    int32_t n_det;        /* 1 .. PE_MAX_DET */
    int64_t n_bins;       /* K >= 1 */
    double f_lo, df;      /* Hz; f_lo > 0, df > 0 */
    int32_t data_dtype;   /* pe_data_dtype_t: complex128 or complex64, interleaved re, im */
    int32_t psd_dtype;    /* pe_psd_dtype_t */
    double strain_scale;  /* stored data = s * physical strain; stored PSD = s^2 * physical PSD */
    int32_t params;       /* pe_params_t */
    int32_t phase;        /* pe_phase_t (4-D requires PE_PHASE_MARG) */
    double amp0;          /* 4-D: physical amplitude A0 of A0 f^-7/6 */
    double gmst;          /* rad */
    double chi_max;       /* prior bound |chi| <= chi_max */
    double dl_max;        /* 11-D prior bound 0 < dL <= dl_max (Mpc) */
    double det_geom[PE_MAX_DET][3];
    int32_t distance;     /* pe_distance_t (a zeroed field: PE_DIST_SAMPLED); PE_DIST_MARG needs 11-D */
    /* Time marginalisation (11-D; zeroed fields: off). time_marg = 1: the
     * likelihood is integrated over tc with a flat prior on [tc_lo, tc_hi]
     * (the paper marginalises the extrinsic parameters, Sec. III):
     *   L_t = (1/T) int_{tc_lo}^{tc_hi} L(theta with tc = t) dt,  T = tc_hi - tc_lo.
     * Every draw is evaluated at tm_points nodes spread evenly over the whole
     * window (theta's own tc is not used), and the integral is the extended
     * trapezoid rule with fourth-order end corrections (weights 17/48, 59/48,
     * 43/48, 49/48 at each end). The spacing h = T / (tm_points - 1) must
     * resolve the likelihood's peak in tc: h at most half its narrowest width
     * 1/sqrt(g_tc,tc) keeps the rule's error far below the split path's for a
     * peak inside the window; a peak that a window edge cuts is integrated to
     * O(h^4). Each call costs tm_points likelihood evaluations per draw.
     * pe_draw sets each draw's tc to its conditional mean under the proposal
     * given the other coordinates and reports the proposal's marginal over tc
     * in logq. */
    int32_t time_marg;
    int32_t tm_points;    /* 8 .. PE_MAX_TM_POINTS */
    double tc_lo, tc_hi;  /* s, tc_lo < tc_hi */
} pe_event_desc_t;

/* Dimension D of theta for a parameter set (4 or 11); 0 if unknown. */
int32_t pe_dim(int32_t params);

/*
 * Create an event: allocate its device tables and prepare them from the data
 * d[n_det][n_bins] and PSD S[n_det][n_bins] (layout as desc says) on `stream`,
 * then synchronise and check the inputs. Prepared per bin: f, f^(1/3),
 * f^(-5/3), ln(f)/3, the folded weights w = 4 df f^(-7/6) d / S (Eq. 1 with
 * the TaylorF2 amplitude), and the prefix sums C_k = sum_{j<k} 4 df f^(-7/3)/S
 * that give (h|h) for any cut. The inputs may be freed after the call.
 * Errors: PE_ERR_ARG (bad desc, S <= 0 or not finite), PE_ERR_NONFINITE (d not
 * finite), PE_ERR_OOM, PE_ERR_HIP. On error *out is NULL.
 */
pe_status_t pe_event_create(const pe_event_desc_t *desc, const void *data_dev, const void *psd_dev, void *stream,
                            pe_event_t *out);

/* Re-prepare an existing event from new data/PSD of the same shape (no
 * allocation; asynchronous). Input errors are reported by pe_event_status. */
pe_status_t pe_event_update(pe_event_t ev, const void *data_dev, const void *psd_dev, void *stream);

/* Synchronise `stream` and return the first error recorded by the event's
 * kernels since the last call (and clear it). */
pe_status_t pe_event_status(pe_event_t ev, void *stream);

/* Pre-size the per-draw workspace for batches of up to max_draws (allocates).
 * pe_loglike_batch grows it on demand otherwise. */
pe_status_t pe_event_reserve(pe_event_t ev, int64_t max_draws);

pe_status_t pe_event_destroy(pe_event_t ev);

/*
 * Metric at theta0 (Sec. II.A: the inner product defines a metric on the
 * waveform manifold): g_ij = sum_d (d_i h_d | d_j h_d) with central
 * differences h(theta0 +- eps_i e_i), the cut frozen at theta0, and the exact
 * derivative i h for the coalescence phase.
 *   theta0_dev : D doubles (device).
 *   fd_step_dev: D doubles (device) or NULL for the default steps (each moves
 *                the phase by ~1e-3 rad at the most sensitive band edge).
 *   flags      : bit0 = do not add the prior precision 12/range^2 on bounded
 *                and periodic coordinates.
 *   g_dev      : D*D doubles, row-major (device). For the marginalised
 *                likelihood the phase direction is projected out (Schur
 *                complement); in 11-D its row and column are then zero before
 *                the prior precision is added. PE_DIST_MARG events project out
 *                dL the same way (jointly with the phase if both are).
 */
pe_status_t pe_metric(pe_event_t ev, const double *theta0_dev, const double *fd_step_dev, int32_t flags,
                      double *g_dev, void *stream);

/*
 * n draws from N(theta0, g^-1) (the proposal of App. A.3, centred on theta0
 * with the metric as precision). Normals come from Philox4x32-10 (Salmon et
 * al., SC'11) with key (seed lo, seed hi) and counter (i lo, i hi, pair j,
 * stream_id), two 53-bit uniforms per block, Box-Muller. Periodic coordinates
 * are wrapped; logq is the log-density of the wrapped Gaussian (sum over the
 * images -2 .. +2 of each periodic coordinate about theta0 wrapped into
 * [0, P)). logprior is the log prior
 * (flat in Mc, eta or q, spins, tc, ra, psi, phic; cos dec; sin iota; dL^2;
 * unnormalised) or -inf outside the support.
 *   theta0_dev: D doubles; g_dev: D*D doubles (device).
 *   theta_dev: [D][n]; logq_dev, logprior_dev: [n] (device, caller-owned).
 * If g is not positive definite every draw is theta0 with logprior = -inf and
 * pe_event_status reports PE_ERR_SINGULAR.
 * PE_DIST_MARG events: dL is first decoupled (g replaced by the Schur
 * complement of its dL row and column, g_dLdL kept), which leaves the
 * distribution of the other coordinates unchanged; logq is the log-density of
 * the proposal's marginal over those coordinates, and logprior has neither the
 * dL^2 factor nor the dL bound. The drawn dL is not used by the likelihood.
 */
pe_status_t pe_draw(pe_event_t ev, const double *theta0_dev, const double *g_dev, uint64_t seed, uint32_t stream_id,
                    int64_t n, double *theta_dev, double *logq_dev, double *logprior_dev, void *stream);

/*
 * Log-density of a mixture of pe_draw's proposals at given points (the paper
 * proposes from a mixture of local proposals, each weighted by its share of
 * the posterior, Sec. II.A; here the components are wrapped Gaussians in the
 * local metric, e.g. the proposals of successive refinement rounds, Sec. III.A):
 *   logq_dev[i] = ln sum_k pi_k q_k(theta_i),  pi_k = weights[k] / sum weights,
 * q_k the density pe_draw reports for draws from (theta0_k, g_k): the wrapped
 * Gaussian summed over the images -2 .. +2 of each periodic coordinate about
 * theta0_k wrapped into [0, P), the event's marginalised coordinates (dL of
 * PE_DIST_MARG events, tc of time-marginalised events, phic of 11-D
 * phase-marginalised events) left out as pe_draw leaves them out. Draws from the
 * mixture are pe_draw calls, one per component (any split of the n draws over
 * the components, e.g. n pi_k each: stratified), with this log q in place of
 * each call's own (the balance heuristic of multiple importance sampling).
 *   weights: m doubles (HOST), finite, >= 0, positive sum; m in 1..PE_MIX_MAX.
 *   theta0_dev [m][D], g_dev [m][D*D] (device): centres and metrics.
 *   theta_dev [D][n] (device): the points, as pe_draw returns them (periodic
 *   coordinates in [0, P); they are not wrapped again).
 *   logq_dev [n] (device, caller-owned).
 * Errors: PE_ERR_ARG (bad m, weights, pointers, n), PE_ERR_HIP. If a component's
 * g is not positive definite, logq is NaN and pe_event_status reports
 * PE_ERR_SINGULAR. The components' factors live in the event (one set per
 * event): calls on one event must not overlap.
 */
pe_status_t pe_mixture_logq(pe_event_t ev, int32_t m, const double *weights, const double *theta0_dev,
                            const double *g_dev, const double *theta_dev, int64_t n, double *logq_dev, void *stream);

/*
 * Log-likelihood ratio (Eq. 3) of n draws. Per draw and detector the kernel
 * reduces Z_d = sum_{k < kcut} conj(w_k) exp(-i Phi_d(f_k)) with
 * Phi_d = Psi(f) + 2 pi f (tc + dt_d) evaluated in FP64, then
 * Z = sum_d R_d Z_d, H = sum_d |R_d|^2 C_{d,kcut} and
 * ln L = Re Z - H/2 (explicit) or ln I0(|Z|) - H/2 (marginalised).
 *   precision: PE_PREC_FP64 (every step in FP64) or PE_PREC_SPLIT (phase in
 *              FP64; reduced-phase sincos, products and sums over blocks of
 *              16 bins in FP32, the block sums accumulated in FP64; final
 *              combination in FP64). The split path bounds each draw's error
 *              from the hardware sine/cosine's measured error spectrum and
 *              the data's noise statistics (taken when the event's tables are
 *              prepared), and re-evaluates in FP64 (same plan, same value as
 *              PE_PREC_FP64) every draw whose bound exceeds the budget of
 *              pe_set_split_guard; pe_loglike_counts reports how many.
 *   loglike_dev: [n]; out-of-support draws get -inf.
 *   aux_dev: NULL or [n][3] = Re Z, Im Z, H (zeros out of support).
 * PE_DIST_MARG events: Z and H are those at the reference distance dl_max
 * (theta's dL is ignored), and with x = dl_max / dL, b = H/2,
 *   ln L = ln int_1^inf 3 x^-4 exp(phi(x) - b x^2) dx,
 * the likelihood integrated over the dL^2 prior on (0, dl_max]; phi = Re(Z) x
 * (explicit phase) or ln I0(|Z| x) (marginalised phase). Evaluated per draw in
 * FP64 by 16-point Gauss-Legendre panels walked outward from the integrand's
 * peak until it falls below e^-45 of its maximum.
 */
pe_status_t pe_loglike_batch(pe_event_t ev, const double *theta_dev, int64_t n, int32_t precision, double *loglike_dev,
                             double *aux_dev, void *stream);

/*
 * Log-likelihood ratios (Eq. 3) of several events' draws in one batch: event e
 * evaluates its n[e] draws theta_dev[e] into loglike_dev[e] (and aux_dev[e] if
 * aux_dev and aux_dev[e] are not NULL), exactly as pe_loglike_batch would
 * (same layouts, same results bit for bit, independent of the other events in
 * the batch). Events of equal n_det share one set of launches (the batch
 * costs a fixed number of launches per detector count, whatever its size),
 * so many small events fill the GPU together (the per-event analyses of
 * Sec. 4 are independent). Each event may appear once. Like pe_loglike_batch,
 * work on an event must not overlap other work on the same event (other
 * streams, other threads): such calls race.
 * n_events: 0 .. 65535; events, theta_dev, n, loglike_dev (and aux_dev if not
 * NULL): host arrays of n_events entries; the pointers in them are device
 * pointers as in pe_loglike_batch. Entries with n[e] = 0 are skipped.
 * Errors: PE_ERR_ARG (bad arrays, duplicate event, bad n or precision),
 * PE_ERR_OOM, PE_ERR_HIP.
 */
pe_status_t pe_loglike_multi(int32_t n_events, const pe_event_t *events, const double *const *theta_dev,
                             const int64_t *n, int32_t precision, double *const *loglike_dev, double *const *aux_dev,
                             void *stream);

/*
 * The whole path for a batch of events in one call: for every item, the
 * stages selected in `stages` run in the order
 *   PE_STAGE_PREP    re-prepare the event's tables from data/psd (as pe_event_update)
 *   PE_STAGE_METRIC  g = metric at theta0 (as pe_metric with fd_step, metric_flags)
 *   PE_STAGE_DRAW    n draws from N(theta0, g^-1) (as pe_draw with seed, stream_id)
 *   PE_STAGE_LOGLIKE ln L of the n draws in theta (as pe_loglike_batch)
 *   PE_STAGE_WEIGHTS weights and ESS of loglike, logprior, logq (as pe_weights_ess)
 * and each stage is one set of launches over all items (events of any
 * detector count and size mixed), so a batch costs a fixed number of launches
 * whatever the number of events. Every item's results equal those of the
 * corresponding single-event calls bit for bit, whatever else is in the batch.
 * Pointers in the items are device pointers with the layouts of the
 * single-event calls; fields of unselected stages are ignored. Each event may
 * appear once. Work on an event must not overlap other work on it.
 * Errors: PE_ERR_ARG (bad item, duplicate event, bad stages or precision),
 * PE_ERR_OOM, PE_ERR_HIP.
 */
#define PE_STAGE_PREP 1
#define PE_STAGE_METRIC 2
#define PE_STAGE_DRAW 4
#define PE_STAGE_LOGLIKE 8
#define PE_STAGE_WEIGHTS 16
#define PE_STAGE_ALL 31

typedef struct {
    pe_event_t ev;
    const void *data, *psd;     /* PREP: [n_det][n_bins] in the event's storage types */
    const double *theta0;       /* METRIC, DRAW: [D] */
    const double *fd_step;      /* METRIC: NULL = default steps */
    int32_t metric_flags;       /* METRIC: as pe_metric */
    uint32_t stream_id;         /* DRAW */
    uint64_t seed;              /* DRAW */
    double *g;                  /* METRIC writes, DRAW reads: [D*D] */
    int64_t n;                  /* DRAW, LOGLIKE, WEIGHTS: draws */
    double *theta;              /* DRAW writes, LOGLIKE reads: [D][n] */
    double *logq, *logprior;    /* DRAW writes, WEIGHTS reads: [n] */
    double *loglike;            /* LOGLIKE writes, WEIGHTS reads: [n] */
    double *aux;                /* LOGLIKE: NULL or [n][3] */
    double *w;                  /* WEIGHTS: NULL or [n] */
    double *stats;              /* WEIGHTS: [4] */
} pe_batch_item_t;

pe_status_t pe_batch_run(int32_t n_items, const pe_batch_item_t *items, int32_t stages, int32_t precision,
                         void *stream);

/*
 * Importance weights (Eq. 5) and ESS (Eq. 6) of n draws, with
 * ln w_i = loglike_i + logprior_i - logq_i and max-shifted sums in FP64.
 *   w_dev: NULL or [n] normalised weights (sum 1; 0 where ln w = -inf).
 *   stats_dev: 4 doubles = {ESS, ln Z = ln mean(w), max ln w, number of
 *              finite ln w}. With no finite ln w: {0, -inf, -inf, 0}.
 * A NaN or +inf ln w (no weight is defined for it) makes ESS, ln Z, max ln w
 * and every w NaN; stats_dev[3] still counts the finite ones.
 * Needs no event; three launches (per-block sums, per-event combine,
 * normalisation).
 */
pe_status_t pe_weights_ess(const double *loglike_dev, const double *logprior_dev, const double *logq_dev, int64_t n,
                           double *w_dev, double *stats_dev, void *stream);

/*
 * pe_weights_ess for callers that cannot allocate device or pinned memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, same kernels and results bit for bit, but the
 * stage's batch record and per-block partial sums live in a fixed scratch
 * array in the library's device memory (about 130 KB per GPU, held until the
 * process ends) instead of buffers the library allocates on first use. The
 * call only enqueues kernels on `stream`; it calls no allocator. Every call on
 * a GPU shares that GPU's scratch, so calls that overlap on one GPU (other
 * streams, other threads) race; calls ordered on one stream do not.
 * Errors: PE_ERR_ARG (n < 0, n > 2^24 (the scratch's limit), NULL pointers),
 * PE_ERR_HIP.
 */
pe_status_t pe_weights_ess_noalloc(const double *loglike_dev, const double *logprior_dev, const double *logq_dev,
                                   int64_t n, double *w_dev, double *stats_dev, void *stream);

/*
 * Model waveform of one parameter point on the event grid, FP64:
 * h_dev[d][k] = s R_d f_k^(-7/6) exp(-i Phi_d(f_k)) for f_k < f_isco, else 0,
 * interleaved complex128. If psd_dev is not NULL (layout as desc), also writes
 * snr2_dev[0] = sum_d (h_d|h_d). No event needed; used to make injections.
 */
pe_status_t pe_waveform(const pe_event_desc_t *desc, const double *theta_dev, const void *psd_dev, double *h_dev,
                        double *snr2_dev, void *stream);

/*
 * Proposal update between rounds of importance sampling (Sec. III.A, end of
 * the efficiency discussion: the proposal is refined iteratively from the
 * local metric around the sampled points). The new centre is the weighted
 * mean of the draws, the weighted covariance about it is returned for
 * diagnostics; the proposal at the new centre is the metric there
 * (pe_metric). Offsets from the current centre take each periodic
 * coordinate (ra, psi, phic) to its image nearest theta0:
 *   d_i = theta_i - theta0,  d -> d - P floor(d/P + 1/2)
 *   m = sum_i w_i d_i / sum_i w_i,   theta0_out = theta0 + m (periodic
 *       coordinates wrapped into [0, P))
 *   cov = sum_i w_i d_i d_i^T / sum_i w_i - m m^T
 * Draws with w_i = 0 are skipped (their parameters are not read into the
 * sums); weights need not be normalised (pe_weights_ess's w is fine). With no
 * positive weight theta0_out = theta0 and cov = 0. Sums in FP64, reduced in a
 * fixed order (bitwise reproducible).
 *   theta_dev [D][n], w_dev [n] (finite, >= 0), theta0_dev [D] (device).
 *   theta0_out_dev [D] (may equal theta0_dev); cov_dev NULL or [D*D] row-major.
 * Errors: PE_ERR_ARG (NULL pointers, n < 0), PE_ERR_OOM, PE_ERR_HIP.
 */
pe_status_t pe_proposal_update(pe_event_t ev, const double *theta_dev, const double *w_dev, int64_t n,
                               const double *theta0_dev, double *theta0_out_dev, double *cov_dev, void *stream);

/*
 * Iterative proposal refinement: `rounds` rounds of
 *   g = pe_metric(theta0); n draws (seed, stream_id = round); ln L (precision);
 *   weights and ESS into stats_dev[4 r .. 4 r + 3]; theta0 = pe_proposal_update(...)
 * followed by g = pe_metric(theta0) at the final centre. Everything is
 * enqueued on `stream` (no host synchronisation). On return theta0_dev holds
 * the refined centre and g_dev the metric there; the buffers hold the last
 * round's draws (from the proposal before the last update).
 *   theta0_dev [D] (in/out), g_dev [D*D] (out), theta_dev [D][n],
 *   logq_dev, logprior_dev, loglike_dev, w_dev [n], stats_dev [rounds][4]
 *   (all device, caller-owned). rounds 1..64.
 * Errors: as the calls it makes; PE_ERR_ARG for rounds out of range.
 */
pe_status_t pe_refine(pe_event_t ev, double *theta0_dev, double *g_dev, int32_t rounds, int64_t n, uint64_t seed,
                      int32_t precision, double *theta_dev, double *logq_dev, double *logprior_dev,
                      double *loglike_dev, double *w_dev, double *stats_dev, void *stream);

/*
 * Tile-mixture proposal (Sec. II.A: tile the metric space, give each tile the
 * part of the prior volume closest to its template, and propose from the
 * tiles in proportion to that volume times the posterior at the template;
 * App. A: template bank, tiling of the prior volume, proposal). Built on the
 * slice of the prior that a detection points to: the ball |y| <= radius in
 * the whitened coordinates y = L^T (theta_S - centre_S) of a metric G = L L^T
 * over the sliced coordinates S. Bank and assignment work in y, where the
 * metric distance is Euclidean. S is every coordinate (sub_mask 0) or, for
 * 11-D events, the four coordinates whose bits are set in sub_mask, in index
 * order (Sec. III tiles the intrinsic parameters, e.g. 0xF = Mc, q, chi1z,
 * chi2z; the others stay at the centre and pe_tile_extrinsic draws them).
 */
typedef struct {
    double centre[PE_MAX_DIM];              /* first D entries used */
    double chol[PE_MAX_DIM * PE_MAX_DIM];   /* L, lower triangular, S x S row-major in the first S*S entries */
    double radius;
    uint32_t sub_mask;                      /* 0: all D coordinates; else 4 bits below bit 11 (11-D only) */
} pe_slice_t;

/*
 * Samples of the slice: candidate i (first .. first + n - 1) has
 * y_a = radius (2 u_a - 1) (a < S), u_a the (a mod 2)-th uniform of Philox
 * block (seed, stream_id, i, a / 2) (as pe_draw's generator); it is kept when
 * |y|^2 <= radius^2 and theta (the centre, plus L^-T y on the sliced
 * coordinates) lies in the prior's support. Kept candidates are written in
 * candidate order: y_dev [S][n], theta_dev [D][n] (row stride n),
 * logprior_dev [n] (the event's log prior); their number goes to count_dev[0]
 * (int64, device). The arithmetic of a candidate is done without
 * contractions, so it is the same bit for bit on every run.
 * Errors: PE_ERR_ARG, PE_ERR_OOM, PE_ERR_HIP.
 */
pe_status_t pe_slice_sample(pe_event_t ev, const pe_slice_t *slice, uint64_t seed, uint32_t stream_id, int64_t first,
                            int64_t n, double *y_dev, double *theta_dev, double *logprior_dev, int64_t *count_dev,
                            void *stream);

/*
 * Stochastic template bank in the slice (App. A, template bank generation):
 * candidates of the slice (as pe_slice_sample with stream_id, counters from
 * 0 in batches of `batch`) are taken in order, and a kept candidate becomes a
 * template when |y - y_t|^2 >= min_dist^2 for every template t so far. Stops
 * after the first batch that adds fewer than stop_fraction times its kept
 * candidates, at max_tiles templates, or after max_batches batches.
 * Templates: tiles_y_dev [S][max_tiles], tiles_theta_dev [D][max_tiles] (row
 * stride max_tiles); *n_tiles and *consumed (candidates drawn) are host
 * outputs.
 * Synchronises the stream (the acceptance runs batch by batch).
 */
pe_status_t pe_tile_bank(pe_event_t ev, const pe_slice_t *slice, double min_dist, uint64_t seed, uint32_t stream_id,
                         int32_t batch, int32_t max_tiles, double stop_fraction, int32_t max_batches,
                         double *tiles_y_dev, double *tiles_theta_dev, int32_t *n_tiles, int64_t *consumed,
                         void *stream);

/*
 * Tile of each sample (App. A, tiling the prior volume): the template nearest
 * in whitened coordinates, |y_s - y_t|^2 summed in index order without
 * contractions; the lowest index among equals.
 *   tiles_y_dev [dim][ld_tiles] (n_tiles used), y_dev [dim][ld_y] (n used),
 *   tile_of_dev [n] int32 (device). n_tiles 1 .. 2^24.
 */
pe_status_t pe_tile_assign(int32_t dim, int32_t n_tiles, const double *tiles_y_dev, int64_t ld_tiles, int64_t n,
                           const double *y_dev, int64_t ld_y, int32_t *tile_of_dev, void *stream);

/*
 * Tile of each sample by waveform similarity (App. A maps the prior volume to
 * the template nearest in match; Sec. III takes the plain overlap for aligned
 * spins): among the sample's n_cand (1, 2, 4 or 8) nearest templates in
 * whitened coordinates, the one of largest match
 *   m(s, t) = |sum_k W_k exp(2 pi i (Psi_s(f_k) - Psi_t(f_k)))| / sqrt(P_s P_t),
 * the overlap maximised over a constant phase and normalised: W_k =
 * sum_d w_d pw_dk with pw = 4 df f^(-7/3) / S from the event's tables and w_d =
 * |R_d|^2 / sum_e |R_e|^2 the detector's share of the sample's response power
 * (one detector: 1), the sum over the bins below both points' cuts, P a
 * point's sum_d w_d (sum of pw_d below its cut), Psi the phase in turns with its
 * 2 pi f tc term (FP64 phases and sine/cosine). The lowest template index among
 * equal matches.
 *   4-D parameter set: one detector; tiles_y_dev, tiles_theta_dev [4][ld_tiles]
 *   (n_tiles used); y_dev, theta_dev [4][ld] (n used).
 *   11-D set: tiles over the intrinsic coordinates (a slice with a 4-bit
 *   sub_mask); the templates and samples share the other coordinates (the
 *   slice's centre), so the responses and delays are common and m is the
 *   network overlap of the two waveforms; tiles_y_dev, y_dev [4][..] (the
 *   sliced coordinates), tiles_theta_dev [11][ld_tiles], theta_dev [11][ld].
 * Outputs tile_of_dev [n] int32 and, if not NULL, match_dev [n] (the chosen
 * template's match). Allocates its scratch and synchronises the stream.
 * Errors: PE_ERR_ARG (a 4-D event with more than one detector, bad sizes,
 * NULL), PE_ERR_OOM, PE_ERR_HIP.
 */
pe_status_t pe_tile_assign_match(pe_event_t ev, int32_t n_tiles, const double *tiles_y_dev,
                                 const double *tiles_theta_dev, int64_t ld_tiles, int64_t n, const double *y_dev,
                                 const double *theta_dev, int64_t ld, int32_t n_cand, int32_t *tile_of_dev,
                                 double *match_dev, void *stream);

/*
 * pe_tile_assign_match with the match maximised over time shifts as well (App.
 * A takes the overlap maximised over the extrinsic time and phase; for tiles
 * over the 11-D set's intrinsic coordinates tc is one of the shared extrinsic
 * coordinates):
 *   m(s, t) = max_j |sum_k W_k exp(2 pi i (Psi_s - Psi_t - f_k tau_j))| / sqrt(P_s P_t),
 * tau_j = j dt, j = -n_shift .. n_shift (the template moved in time by tau_j).
 * dt > 0 (seconds), n_shift 1 .. 4096; match_dev is required; n_cand as for
 * pe_tile_assign_match (0: every template). Costs about (2 n_shift + 1) / 8
 * walks over the bins per candidate. Errors as pe_tile_assign_match.
 */
pe_status_t pe_tile_assign_match_shift(pe_event_t ev, int32_t n_tiles, const double *tiles_y_dev,
                                       const double *tiles_theta_dev, int64_t ld_tiles, int64_t n,
                                       const double *y_dev, const double *theta_dev, int64_t ld, int32_t n_cand,
                                       double dt, int32_t n_shift, int32_t *tile_of_dev, double *match_dev,
                                       void *stream);

/*
 * Proposal draws from the tiles (Sec. II.A; App. A, the proposal): sample s
 * (of P) carries the mass m_s = exp(ll_t(s) - max ll + lp_s - max lp) (its
 * tile's template log-likelihood tile_loglike_dev[t(s)] and its log prior
 * sample_logprior_dev[s]; 0 where either is -inf); draw i takes the first
 * uniform u of Philox block (seed, stream_id, i, 0) and returns the smallest
 * s with u C_P <= C_s, C_s = m_0 + ... + m_s (FP64 prefix sums).
 *   theta_dev [D][n] = sample s (samples_theta_dev [D][ld]),
 *   logprior_dev[i] = lp_s, logq_dev[i] = ln m_s - ln(C_P / P) (the proposal
 *   density relative to the flat measure the samples come from),
 *   index_dev[i] = s (int64; may be NULL).
 * With no positive mass every draw gets logprior -inf, logq 0, index -1.
 * Importance weights then follow from pe_weights_ess as for pe_draw.
 */
pe_status_t pe_tile_draw(int32_t n_tiles, const double *tile_loglike_dev, int64_t n_samples,
                         const int32_t *tile_of_dev, const double *sample_logprior_dev, int32_t dim,
                         const double *samples_theta_dev, int64_t ld, uint64_t seed, uint32_t stream_id, int64_t n,
                         double *theta_dev, double *logq_dev, double *logprior_dev, int64_t *index_dev, void *stream);

/*
 * Extrinsic coordinates of tile draws (Sec. III: intrinsic and extrinsic
 * parameters partially decouple, so the prior volume is tiled over the
 * intrinsic ones and the others are proposed apart). theta_dev [D][n] holds
 * draws whose coordinates in sub_mask come from pe_tile_draw on a slice with
 * that sub_mask; every other coordinate is replaced by a draw from the
 * marginal of N(theta0, g^-1) over the coordinates outside sub_mask: the
 * normals of pe_draw (Philox blocks (seed, stream_id, i, pair)), g decoupled
 * at the sub_mask coordinates by the Schur complement as pe_draw decouples the
 * likelihood's marginalised ones (which it treats as pe_draw does: dL of
 * PE_DIST_MARG events and phic of 11-D phase-marginalised events left out of
 * log q, tc of time-marginalised events set to its conditional mean given the
 * composed draw). Then
 *   logq_dev[i] += the log density of that marginal (wrapped Gaussian, images
 *                  -2 .. +2 of each periodic coordinate), so that it holds the
 *                  composed proposal's log density;
 *   logprior_dev[i] = the log prior of the composed draw, or stays -inf where
 *                  it was (draws without a sample).
 *   theta0_dev [D], g_dev [D*D] (device): the metric proposal whose marginal
 *   is taken. sub_mask: nonzero, bits below 11, none of the periodic
 *   coordinates ra, psi, phic (bits 4, 7, 10). 11-D events only.
 * flags: PE_TILE_CONDITIONAL draws the other coordinates from their
 * conditional given each draw's sub_mask coordinates instead (the
 * marginalised ones integrated out): mean theta0_E + C_EI C_II^-1
 * (theta_I - theta0_I), covariance C_EE - C_EI C_II^-1 C_IE with C = g^-1; log
 * q gains that conditional density. sub_mask must then leave out the
 * marginalised coordinates.
 * If g is not positive definite every draw gets logprior -inf (theta and logq
 * as they were) and pe_event_status reports PE_ERR_SINGULAR.
 * Errors: PE_ERR_ARG, PE_ERR_HIP.
 */
#define PE_TILE_CONDITIONAL 1
pe_status_t pe_tile_extrinsic(pe_event_t ev, const double *theta0_dev, const double *g_dev, uint32_t sub_mask,
                              int32_t flags, uint64_t seed, uint32_t stream_id, int64_t n, double *theta_dev,
                              double *logq_dev, double *logprior_dev, void *stream);

/*
 * Tile values for the next round (the iterative update of the proposal that
 * the paper suggests at the end of Sec. III.A, applied to the tile mixture):
 * tile j's posterior mass estimated from the previous round, P_j = the sum of
 * the normalised weights of the draws that came from it, mixed with the
 * previous round's tile probability p_j (defensive share alpha):
 *   pi_j = (1 - alpha) P_j / sum P + alpha p_j,
 *   p_j = exp(l_j - max l) V_j / sum_k exp(l_k - max l) V_k,
 *   V_j = sum over the tile's samples of exp(lp_s - max lp) (prior volume);
 *   out_dev[j] = ln pi_j - ln V_j (-inf where pi_j or V_j is 0).
 * Passed to pe_tile_draw in place of the template log-likelihoods, it gives
 * sample s the mass pi_j exp(lp_s) / V_j.
 *   tile_loglike_dev [n_tiles]: the values the previous pe_tile_draw used;
 *   tile_of_dev, sample_logprior_dev [n_samples] (n_samples <= 2^31);
 *   index_dev [n] (pe_tile_draw's sample indices; negative ones skipped),
 *   w_dev [n] (normalised weights of those draws, pe_weights_ess: each in
 *   [0, 1], sum 1); alpha in [0, 1]; out_dev [n_tiles], not aliasing the input.
 * The per-tile sums are 64-bit fixed point (prior volume in units of 2^-32 of
 * the largest sample's, weights in units of 2^-52), so the result does not
 * depend on the order of the additions.
 */
pe_status_t pe_tile_reweight(int32_t n_tiles, const double *tile_loglike_dev, int64_t n_samples,
                             const int32_t *tile_of_dev, const double *sample_logprior_dev, int64_t n,
                             const int64_t *index_dev, const double *w_dev, double alpha, double *out_dev,
                             void *stream);

/*
 * Relative binning (Zackay, Dai & Venumadhav 2018; the paper lists such
 * reduced representations among the ways to speed the likelihood up, Sec. I).
 * About a fiducial point theta_f near the peak, the ratio rho_d(f) =
 * exp(-i (Phi_d - Phi0_d)(f)) of a draw's phase factor to the fiducial's is
 * smooth in f; it is replaced in each bin by its linear interpolation between
 * the bin edges, so that
 *   Z_d = R_d sum_b [rho_d(f_b) A0_{d,b} + s_{d,b} A1_{d,b}],
 *   s_{d,b} = (rho_d(f_{b+1}) - rho_d(f_b)) / (f_{b+1} - f_b),
 *   A0_{d,b} = sum_{k in b, k < kcut} a_k,  A1_{d,b} = sum_{k in b, k < kcut} a_k (f_k - f_b),
 *   a_k = conj(w_k) exp(-i Phi0_d(f_k))  (w as in pe_loglike_batch),
 * with the bin holding the draw's cut summed only below it; (h|h) stays exact.
 * Edges: grid indices 0 = k_0 < ... < k_B = K; the next edge is the first k
 * where E(f) = 2 pi sum_a sgn(a) (f / f_a)^a (a in {-5/3, -2/3, 1, 5/3, 7/3},
 * f_a = f_lo for a < 0, f_lo + K df for a > 0) has grown by at least eps.
 * pe_relbin_setup computes the edges on the host, then the fiducial phases
 * and the per-bin and prefix sums on the device (it allocates and
 * synchronises); afterwards pe_loglike_batch(..., PE_PREC_RELBIN, ...)
 * evaluates draws at O(bins) cost each. A new setup replaces the previous
 * one; pe_event_update does not refresh it (set up again after new data).
 *   theta_f_dev: D doubles (device). eps > 0 (0 gives one bin per grid
 *   point); at most max_edges edges (PE_ERR_BUDGET beyond).
 * pe_relbin_edges copies the edges to a host array of capacity cap and
 * writes their number to *n (0 before any setup); with edges NULL it writes
 * only the number.
 */
pe_status_t pe_relbin_setup(pe_event_t ev, const double *theta_f_dev, double eps, int32_t max_edges, void *stream);
pe_status_t pe_relbin_edges(pe_event_t ev, int64_t *edges, int32_t cap, int32_t *n);

/* The proposal's uniforms: u_dev[(i*npairs + j)*2 + {0,1}] for draw i and
 * block j < npairs, exactly the values pe_draw uses. */
pe_status_t pe_rng_uniforms(uint64_t seed, uint32_t stream_id, int64_t n, int32_t npairs, double *u_dev,
                            void *stream);

/*
 * Serving loop. A server owns one slab of device memory (hbm_budget bytes), a
 * stream and a native worker thread. Requests (one detection event each:
 * data, PSD, proposal centre, number of draws) are submitted from any thread
 * and queued; the worker admits them in arrival order while their footprint
 * (tables, workspace and per-draw buffers, all in the slab) fits the free
 * memory and fewer than max_active are on the device, and runs for each
 * newly admitted group: table preparation, metric, draws and the
 * log-likelihood prologue as batched launches. The hot loop then runs in
 * slices of about slice_ms: each slice takes draw tiles of the active events,
 * shortest remaining work first, into one work queue, so requests that arrive
 * while others are on the GPU join the next slice and their work overlaps on
 * the device (continuous batching). When an event's last tile is done the
 * same slice combines its partials, computes ln L, the weights and the ESS,
 * and the event's results are copied back and its memory released. With
 * use_graph, the slice (work-queue setup, hot loop, ln L, weights) is
 * captured once in a hipGraph and replayed on the new contents of fixed
 * device buffers. Every result equals that of the single-event calls for the
 * same inputs bit for bit, whatever else is in flight.
 */
typedef struct pe_server_s *pe_server_t;

typedef struct {
    int64_t hbm_budget;  /* bytes of the device slab for admitted requests */
    int32_t precision;   /* PE_PREC_SPLIT or PE_PREC_FP64 */
    int32_t max_active;  /* requests on the device at once, 1..4096 */
    double slice_ms;     /* target duration of one hot-loop slice, > 0 */
    int32_t use_graph;   /* 1: replay the slice as a captured hipGraph */
    int32_t max_groups;  /* cap on an event's groups of frequency chunks (0 = automatic) */
    int32_t items_target;    /* hot-loop plan (see pe_set_plan); 0 = the library's setting */
    int32_t min_group_bins;  /* hot-loop plan (see pe_set_plan); 0 = the library's setting */
} pe_server_config_t;

typedef struct {
    pe_event_desc_t desc;
    const void *data, *psd;  /* [n_det][n_bins] in desc's storage types; valid until the request completes */
    int32_t data_on_host;    /* 1: data and psd are host memory, copied to the slab at admission */
    int32_t metric_flags;    /* as pe_metric */
    const double *theta0;    /* host [D]: proposal centre (copied at submission) */
    uint64_t seed;           /* draws as pe_draw(seed, stream_id) */
    uint32_t stream_id;
    int32_t pad;
    int64_t n_draws;         /* 1 .. 2^22 */
    double *loglike_out;     /* NULL or host [n]: ln L of every draw */
    double *w_out;           /* NULL or host [n]: normalised weights */
    double *theta_out;       /* NULL or host [D][n]: the draws */
} pe_request_t;

typedef struct {
    int64_t ticket;
    int32_t status;      /* PE_OK or the request's error */
    int32_t n_active;    /* requests on the device when this one was admitted */
    double stats[4];     /* as pe_weights_ess: ESS, ln Z, max ln w, finite count */
    double t_submit;     /* seconds on the server clock (pe_server_now) */
    double t_admit;
    double t_done;
} pe_result_t;

/* Start a server (allocates the slab; starts the worker). Errors: PE_ERR_ARG,
 * PE_ERR_OOM, PE_ERR_HIP. */
pe_status_t pe_server_create(const pe_server_config_t *cfg, pe_server_t *out);
/* Queue a request; *ticket identifies it. Host-side argument checks only;
 * a request whose footprint exceeds the whole budget completes with
 * PE_ERR_BUDGET. */
pe_status_t pe_server_submit(pe_server_t srv, const pe_request_t *req, int64_t *ticket);
/* Wait up to timeout_s seconds (< 0: forever) for a request; PE_ERR_TIMEOUT
 * if it has not completed. A result is returned once. */
pe_status_t pe_server_wait(pe_server_t srv, int64_t ticket, double timeout_s, pe_result_t *out);
/* Seconds on the server's monotonic clock. */
double pe_server_now(pe_server_t srv);
/* Counters: {requests completed, slices run, hot-loop items run, graph
 * replays, peak slab bytes in use, admissions waiting for memory}. */
pe_status_t pe_server_counters(pe_server_t srv, int64_t out[6]);
/* Device time so far, in milliseconds, from HIP events on the server's stream:
 * out[0] the hot-loop slices (queue setup, hot loop, ln L, weights), out[1]
 * the admission stages (prep, metric, draws, log-likelihood prologue). Their
 * sum over a window is the server's GPU busy time. */
pe_status_t pe_server_busy(pe_server_t srv, double out[2]);
/* The tile-shape autotuner of the serving loop (the benchmark description asks
 * for tile shapes picked by the project's own autotuner). Groups the n given
 * events into shape buckets (detector count, number of bins rounded up to a
 * power of two), runs pe_autotune_plan on each bucket's events and draws
 * (theta_dev[i]: device [D][n_draws[i]]) on the server's stream in the
 * server's precision, and keeps the fastest plan per bucket: later requests of
 * a tuned bucket are planned with it (over the config's items_target and
 * min_group_bins); other buckets keep the config's or the library's setting.
 * A request's results then equal the single-event calls run under pe_set_plan
 * with its bucket's plan. Call on an idle server (PE_ERR_ARG otherwise: the
 * timings would include other work); the events are the caller's own
 * (pe_event_create) and are left unchanged apart from their workspace.
 * Errors: PE_ERR_ARG, PE_ERR_HIP, PE_ERR_OOM. */
pe_status_t pe_server_tune(pe_server_t srv, int32_t n, const pe_event_t *events, const double *const *theta_dev,
                           const int64_t *n_draws, int32_t reps);
/* The tuned plans: *count buckets; the first min(max, *count) as out[4 i ..]
 * = {n_det, log2 of the bucket's bin bound, items_target, min_group_bins} and,
 * if ms is not NULL, ms[i] = the tuning batch's milliseconds with that plan. */
pe_status_t pe_server_plans(pe_server_t srv, int32_t max, int32_t *out, double *ms, int32_t *count);
/* Finish every submitted request, stop the worker, free the slab. */
pe_status_t pe_server_destroy(pe_server_t srv);

/* Kernel timing with HIP events on the launch stream. enable != 0 starts
 * recording around the hot-loop kernel launches; pe_profile_read synchronises
 * the recorded events and returns the summed milliseconds and launch count of
 * the named kernel ("loglike_split", "loglike_fp64"), then clears it. */
pe_status_t pe_profile_enable(int32_t enable);
pe_status_t pe_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/* Budget of the split path's per-draw error bound, |d ln L| (default 5e-4,
 * half the split path's stated 1e-3): draws whose bound exceeds it are
 * re-evaluated in FP64 within the same call. 0 re-evaluates every live draw
 * (the result then equals PE_PREC_FP64 bit for bit); +inf never does. Global
 * setting, read at launch time. Errors: PE_ERR_ARG (negative or NaN). */
pe_status_t pe_set_split_guard(double budget);
pe_status_t pe_get_split_guard(double *budget);

/* Counts of the event's last log-likelihood batch (pe_loglike_batch,
 * pe_loglike_multi, pe_batch_run): out[0] = in-support draws, out[1] = draws
 * the split path re-evaluated in FP64 (0 for PE_PREC_FP64). Synchronises
 * `stream`. Errors: PE_ERR_ARG (NULL), PE_ERR_HIP. */
pe_status_t pe_loglike_counts(pe_event_t ev, int64_t out[2], void *stream);

/* Work split of the hot loop: draws per tile are fixed (256); n_chunks caps
 * the number of groups of frequency chunks one event's tile is spread over
 * (0 = automatic, at most 64; 1 = one group walks the whole band). Results do
 * not depend on it. Global setting, read at launch time. */
pe_status_t pe_set_chunks(int32_t n_chunks);

/* Plan of the hot loop's work decomposition, read at launch time (global):
 * each event's tiles x groups aim at about items_target work items (more
 * items balance the persistent queues better; fewer write fewer partials),
 * with at least min_group_bins bins per group. Defaults 16384 and 1024.
 * Results are bitwise reproducible for a fixed setting and change only in
 * rounding between settings. Errors: PE_ERR_ARG (out of range). */
pe_status_t pe_set_plan(int32_t items_target, int32_t min_group_bins);
pe_status_t pe_get_plan(int32_t *items_target, int32_t *min_group_bins);

/* Autotuner of the plan for a workload: times pe_loglike_multi on the given
 * events and draws (one untimed and `reps` timed batches per candidate, HIP
 * events on `stream`) over items_target in {4096 .. 65536} and min_group_bins
 * in {256 .. 4096}, and returns the fastest pair and its time per batch in
 * milliseconds. The library's setting is left unchanged; apply the result with
 * pe_set_plan (or a server's config). Allocates scratch for the log-likelihoods
 * and synchronises `stream`. */
pe_status_t pe_autotune_plan(int32_t n_events, const pe_event_t *events, const double *const *theta_dev,
                             const int64_t *n, int32_t precision, int32_t reps, int32_t *best_items_target,
                             int32_t *best_min_group_bins, double *best_ms, void *stream);

const char *pe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
