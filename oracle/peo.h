/*
 * peo.h -- plain FP64 CPU oracle for metric-based importance sampling of
 * compact-binary gravitational-wave signals (Nitz, arXiv:2410.05190).
 *
 * THIS IS TEST INFRASTRUCTURE. It exists only to check the GPU library
 * against the paper's definitions. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it. The GPU library never
 * includes, links or calls anything here, and this file includes nothing
 * of the GPU library: the two implement the same definitions independently.
 *
 * Every quantity is evaluated the slow, obvious way, in double precision:
 *   - noise-weighted inner product (Sec. II.A, Eq. 1), left-point sum on the
 *     half-open grid f_k = f_lo + k*df, k = 0..K-1;
 *   - log-likelihood ratio against noise (Sec. II.A, Eq. 3), optionally
 *     marginalised over the coalescence phase with a uniform prior;
 *   - importance weights (App. A.3, Eq. 5) and effective sample size (Eq. 6);
 *   - the waveform-manifold metric (Sec. II.A, the metric induced by the
 *     inner product) as the Fisher matrix of the network waveform.
 * The waveform model is TaylorF2 (stationary-phase inspiral, 3.5PN phase,
 * aligned spins, Newtonian amplitude) cut at the test-mass ISCO frequency of
 * the total mass; the paper itself uses IMRPhenom models, which are not
 * available here.
 *
 * Units: masses in solar masses (detector frame), distance in Mpc, times in
 * seconds, angles in radians. Stored data and PSD may carry a unit scale s:
 * data = s * physical strain, psd = s^2 * physical PSD; inner products are
 * invariant, the model waveform is multiplied by s.
 */
#ifndef PEO_H
#define PEO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PEO_MAX_DET 4
#define PEO_MAX_DIM 11

/* parameter sets */
#define PEO_PARAMS_4D 0  /* Mc, eta, chi_eff, tc ; fixed real amplitude amp0, one response */
#define PEO_PARAMS_11D 1 /* Mc, q, chi1z, chi2z, ra, dec, iota, psi, dL, tc, phic */
/* likelihood forms */
#define PEO_PHASE_MARG 0     /* ln I0(|Z|) - H/2, coalescence phase marginalised */
#define PEO_PHASE_EXPLICIT 1 /* Re Z - H/2 */
/* distance treatment (11-D only) */
#define PEO_DIST_SAMPLED 0 /* dL is a sampled coordinate of theta */
#define PEO_DIST_MARG 1    /* the likelihood is marginalised over dL with the dL^2 prior on (0, dl_max] */

typedef struct {
    int n_det;
    long n_bins;
    double f_lo, df;
    const double *data; /* [n_det][n_bins][2] (re, im); NULL for template-only use */
    const double *psd;  /* [n_det][n_bins] */
    double strain_scale;
    int params;
    int phase;
    double amp0;    /* 4-D only: physical amplitude A0 of A0 f^-7/6 */
    double gmst;    /* rad */
    double chi_max; /* |chi| bound of the prior */
    double dl_max;  /* Mpc, upper bound of the distance prior (11-D) */
    double det_geom[PEO_MAX_DET][3]; /* latitude, longitude, x-arm azimuth (from north to east) */
    int distance;   /* PEO_DIST_SAMPLED or PEO_DIST_MARG */
    int time_marg;  /* 11-D: 1 = the likelihood is marginalised over tc with a flat prior on [tc_lo, tc_hi] */
    double tc_lo, tc_hi;
} peo_event;

/* Per-draw source quantities derived from theta. */
typedef struct {
    int in_support;
    double mc, M, eta, delta, chi1, chi2;
    double tc, phic;
    double rre[PEO_MAX_DET], rim[PEO_MAX_DET]; /* complex response incl. amplitude and scale */
    double dt[PEO_MAX_DET];                     /* arrival delay w.r.t. geocentre, s */
    double fisco;
    long kcut; /* -1 until a caller computes it */
    double phi[8], phil[8]; /* TaylorF2 coefficients */
} peo_source;

int peo_dim(int params);
double peo_t_sun(void);
double peo_mpc_m(void);
double peo_c_si(void);
double peo_r_earth(void);

/* TaylorF2 coefficients phi_j and log coefficients phil_j, j = 0..7, of
 * Psi = 2 pi f tc - phic - pi/4 + 3/(128 eta v^5) sum_j (phi_j + phil_j ln v) v^j.
 * delta = (m1 - m2)/M, chi1/chi2 aligned spins of the heavier/lighter body. */
void peo_pn_coeffs(double eta, double delta, double chi1, double chi2, double phi[8], double phil[8]);
/* Phase Psi(f) in radians of the source (no detector delay). */
double peo_psi(const peo_source *s, double f);
double peo_f_isco(double M);
long peo_kcut(const peo_event *ev, double fisco);
void peo_antenna(const double geom[3], double ra, double dec, double psi, double gmst,
                 double *fplus, double *fcross, double *dt);
/* theta: D contiguous values. Returns in_support. Always fills s. */
int peo_source_from_theta(const peo_event *ev, const double *theta, peo_source *s);

/* h[d][k][2] for k < n_bins (zero above the cut) at theta, physical*scale units.
 * kcut_override < 0 uses the draw's own cut. */
void peo_waveform(const peo_event *ev, const double *theta, long kcut_override, double *h);
/* 4 df Re sum_k conj(a_k) b_k / S_k over all bins of detector d. */
double peo_inner(const peo_event *ev, int d, const double *a, const double *b);

double peo_log_i0(double x);

/*
 * Distance marginalisation (Sec. III: the extrinsic parameters are marginalised
 * with analytic or numerical formulas; for the distance, the integral over the
 * dL^2 prior of Singer & Price 2016). With Z and H evaluated at the reference
 * distance dl_max, the likelihood at distance dL is Z x and H x^2 with
 * x = dl_max / dL, and
 *   L_D = int_0^dl_max (3 dL^2 / dl_max^3) L(dL) ddL = int_1^inf 3 x^-4 exp(phi(x) - b x^2) dx,
 * phi(x) = a x (explicit phase, a = Re Z) or ln I0(a x) (marginalised phase,
 * a = |Z|), b = H / 2. Returns ln L_D.
 */
double peo_log_dist_marg(double a, double b, int explicit_phase);

/* theta: [D][n] (row j holds parameter j of every draw). zh: [n][3] = Re Z, Im Z, H, may be NULL.
 * Out-of-support draws get -inf. n_threads <= 0: OpenMP default. Distance-marginalised events:
 * Z and H at the reference distance dl_max (the draw's dL is not used), ln L = ln L_D. */
void peo_loglike(const peo_event *ev, const double *theta, long n, double *loglike, double *zh, int n_threads);

/* Default finite-difference steps at theta0 (D values). */
void peo_default_steps(const peo_event *ev, const double *theta0, double *steps);
/* Fisher metric. flags: bit0 = do not add the prior regularisation,
 * bit1 = raw (no coalescence-phase projection, 4-D returns 5x5 with phic last).
 * Distance-marginalised events also project out dL (Schur complement; its row and
 * column are zero apart from the regularisation on the diagonal).
 * g is (D or D+1)^2 row-major. Returns 0. */
int peo_metric_fd(const peo_event *ev, const double *theta0, const double *steps, int flags, double *g);

/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11). */
void peo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* u[i*2*npairs + 2j + {0,1}] = the two 53-bit uniforms of block (i, j). */
void peo_uniforms(uint64_t seed, uint32_t stream, long n, int npairs, double *u);
/* Draws from N(theta0, g^-1), periodic coordinates wrapped. theta [D][n]. Returns 0, or 3 if
 * g is not positive definite. logq uses the image sum over the wrapped coordinates.
 * Distance-marginalised events: dL is decoupled first (g replaced by the Schur complement of
 * its dL row and column, g_dLdL kept), which leaves the distribution of the other coordinates
 * unchanged; logq is then the log of the proposal's marginal density over those coordinates,
 * and the prior has no dL factor and no dL bound: the drawn dL is never used. */
int peo_draw(const peo_event *ev, const double *theta0, const double *g, uint64_t seed, uint32_t stream,
             long n, double *theta, double *logq, double *logprior);
/* Proposal log-density of wrapped draws from theta alone (quadratic-form route). */
int peo_logq_theta(const peo_event *ev, const double *theta0, const double *g, const double *theta,
                   long n, double *logq);
/* Log-density of the mixture sum_m pi_m q_m of the wrapped metric Gaussians
 * (theta0 [m][D], g [m][D*D]) with pi_m = weights_m / sum weights; q_m as in
 * peo_logq_theta. Returns 0, -1 for bad weights, else a component's code. */
int peo_mixture_logq(const peo_event *ev, int m, const double *weights, const double *theta0, const double *g,
                     const double *theta, long n, double *logq);
double peo_logprior(const peo_event *ev, const double *theta);

/* stats = {ESS, lnZ, max log w, n_in_support}. w may be NULL. */
void peo_weights_ess(const double *loglike, const double *logprior, const double *logq, long n,
                     double *w, double *stats);

/* Slice of the prior: the ball |y| <= radius in whitened coordinates
 * y = L^T (theta_S - centre_S), G = L L^T (chol: row-major lower L, S x S) over
 * the sliced coordinates S: all D when sub_mask is 0, else those whose bit is
 * set in sub_mask (in index order); the other coordinates stay at the centre
 * (Sec. III tiles the intrinsic coordinates alone). */
typedef struct {
    double centre[PEO_MAX_DIM];
    double chol[PEO_MAX_DIM * PEO_MAX_DIM];
    double radius;
    unsigned sub_mask;
} peo_slice;

/* Number of sliced coordinates and their indices. */
int peo_slice_dims(const peo_event *ev, const peo_slice *sl, int *idx);

/* Extrinsic coordinates of tile draws (Sec. III: intrinsic and extrinsic
 * parameters partially decouple, so the prior volume is tiled over the former
 * and the latter are proposed apart): theta [D][n] holds draws whose
 * coordinates in sub_mask come from the tile mixture; every other coordinate is
 * drawn from the marginal of N(theta0, g^-1) over the coordinates outside
 * sub_mask (and outside the likelihood's marginalised ones), with the normals
 * of peo_draw (Philox blocks (seed, stream, i, pair)) and the metric decoupled
 * at the sub_mask coordinates as at the marginalised ones; logq[i] gains that
 * marginal's log density (wrapped on periodic coordinates); logprior[i]
 * becomes the log prior of the composed draw, or stays -inf. With conditional
 * set, the kept coordinates come instead from their conditional given the
 * draw's sub_mask coordinates (the marginalised ones integrated out), and logq
 * gains that conditional density. Returns 0, or nonzero when g is not positive
 * definite or the mask is not allowed (nothing written then). */
int peo_tile_extrinsic(const peo_event *ev, const double *theta0, const double *g, unsigned sub_mask, int conditional,
                       uint64_t seed, uint32_t stream, long n, double *theta, double *logq, double *logprior);

int peo_slice_candidate(const peo_event *ev, const peo_slice *sl, uint64_t seed, uint32_t stream, uint64_t i,
                        double *y, double *theta);
long peo_slice_sample(const peo_event *ev, const peo_slice *sl, uint64_t seed, uint32_t stream, long first, long n,
                      double *y, double *theta, double *logprior);
long peo_tile_bank(const peo_event *ev, const peo_slice *sl, double min_dist, uint64_t seed, uint32_t stream,
                   long batch, long max_tiles, double stop_fraction, long max_batches, double *ty, double *tth,
                   long *consumed);
void peo_tile_assign(int D, long n_tiles, const double *ty, long ld_t, long n, const double *y, long ld_s,
                     int *tile_of);
/* Waveform match of two points (the overlap maximised over a constant phase,
 * normalised); -1 outside the support. */
double peo_match(const peo_event *ev, const double *theta_a, const double *theta_b);
/* The match maximised over time shifts tau_j = j dt, |j| <= n_shift, as well. */
double peo_match_shift(const peo_event *ev, const double *theta_a, const double *theta_b, double dt, int n_shift);
/* Tile of each sample by the shift-maximised match (brute force). */
void peo_tile_assign_match_shift(const peo_event *ev, long n_tiles, const double *tth, long ld_t, long n,
                                 const double *th, long ld_s, double dt, int n_shift, int *tile_of, double *match);
/* Tile of each sample by largest match (brute force over the templates). */
void peo_tile_assign_match(const peo_event *ev, long n_tiles, const double *tth, long ld_t, long n,
                           const double *th, long ld_s, int *tile_of, double *match);
int peo_tile_draw(long n_tiles, const double *tile_ll, long P, const int *tile_of, const double *lp, int D,
                  const double *samples, long ld, uint64_t seed, uint32_t stream, long n, double *theta,
                  double *logq, double *logprior, long *index);

/* Per-tile values for the next round's peo_tile_draw from the previous round's
 * draws (index) and normalised weights (w), defensive share alpha. */
void peo_tile_reweight(long n_tiles, const double *tile_ll, long P, const int *tile_of, const double *lp, long n,
                       const long *index, const double *w, double alpha, double *out);

/* Relative binning: bin edges from the phase envelope (returns the number of
 * edges or -1), and log-likelihoods of draws about a fiducial point. */
long peo_relbin_edges(const peo_event *ev, double eps, long max_edges, long *edges);
void peo_relbin_loglike(const peo_event *ev, const double *theta_f, long n_edges, const long *edges,
                        const double *theta, long n, double *loglike, double *zh);

/* Weighted centre and covariance of draws about theta0 (proposal update between
 * rounds). theta0_out [D]; cov [D*D] or NULL. Returns the number of w > 0. */
long peo_proposal_update(const peo_event *ev, const double *theta0, const double *theta, long n, const double *w,
                         double *theta0_out, double *cov);

#ifdef __cplusplus
}
#endif
#endif
