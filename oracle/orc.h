/*
 * orc.h -- plain FP64 CPU oracle for Monte-Carlo dust continuum radiative
 * transfer (Robitaille 2011, HYPERION).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this code; it exists so that tests, the smoke check and the
 * CPU baseline leg of the benchmark can judge the HIP path.  It shares no
 * code, header, table or constant generator with the HIP library.
 *
 * Units are cgs throughout.  Arrays are C-ordered with x fastest:
 *     cell index j = i + nx*(jy + ny*k).
 * Frequency bins are ordered by increasing frequency.
 *
 * Parity status per function is stated in orc.c's header comment.
 */
#ifndef ORC_H
#define ORC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_model orc_model;

/* Event record of the per-packet log.  type: 0 EMIT, 1 SCATTER, 2 ABSORB,
 * 3 ESCAPE, 4 KILLED.  cell = cell of the event (for ESCAPE the last cell
 * inside the grid, or the start cell if the packet never entered), nu = the
 * frequency bin after the event, incl = inclination bin (ESCAPE only, else -1). */
typedef struct {
    int64_t packet;
    int32_t index;
    int32_t type;
    int32_t cell[3];
    int32_t nu;
    int32_t incl;
    int32_t reserved;
} orc_event;

typedef struct {
    int64_t n_packets;          /* source packets per Lucy iteration        */
    int64_t n_packets_final;    /* packets of the final binning pass        */
    int32_t n_iter;             /* Lucy iterations of orc_run               */
    uint64_t seed;              /* Philox key word 0 = seed mod 2^32        */
    double t_init;              /* initial temperature [K]                  */
    int64_t max_events;         /* interactions before a packet is killed   */
    double conv_p;              /* percentile of the convergence test (0..1)*/
    double conv_q_thres;
    double conv_d_thres;
    double conv_dT_thres;       /* max |dT/T| threshold                     */
    int32_t stop_on_convergence;
    int32_t source_sampling;    /* 0 luminosity-proportional, 1 equal       */
    int32_t want_noise;         /* accumulate sum of squared weights        */
    int32_t event_log_packets;  /* log events of packets [0, this)          */
    int32_t event_log_cap;      /* events kept per logged packet            */
    int32_t bin_every_iteration;/* bin escapes in the Lucy iterations too   */
    int32_t n_threads;          /* OpenMP threads (0 = default)             */
    int32_t chunk;              /* packets per work chunk (0 = 1024)        */
    double mrw_gamma;           /* modified random walk: step when the sphere
                                   to the nearest cell wall holds at least this
                                   many Rosseland mean free paths (0 = off)  */
} orc_run_cfg;

typedef struct {
    int32_t iteration;          /* index of the iteration just finished     */
    int32_t converged_q;        /* Q < Q_thres and Delta < Delta_thres      */
    int32_t converged_dT;       /* max r over the mask < dT threshold       */
    int32_t pad;
    double q;                   /* p-th percentile of R_j (Eq.5)            */
    double delta;               /* delta(Q^{i-1}, Q^i) (Eq.6)               */
    double max_dT;              /* max over mask of |T^i - T^{i-1}|/T^{i-1} */
    double p999_dT;             /* 99.9th percentile of the same            */
    int64_t n_mask;             /* cells in the dT mask                     */
    int64_t n_r;                /* cells entering the percentile of R       */
    int64_t n_unsampled;        /* dust cells with zero absorption          */
    int64_t n_t_clamped;        /* cells whose T hit the table range        */
    int64_t n_row_clamped;      /* cells whose emission row was clamped     */
    int64_t n_cross_dust;       /* segments walked in cells with rho > 0    */
    int64_t n_cross_empty;      /* segments walked in cells with rho = 0    */
    int64_t n_scatter;
    int64_t n_absorb;
    int64_t n_escape;
    int64_t n_killed;
    double e_escaped;           /* energy of escaped packets [erg]          */
    double e_killed;            /* energy of killed packets [erg]           */
    double seconds;             /* wall time of the transport               */
    int64_t n_mrw;              /* modified-random-walk steps               */
} orc_iter_stats;

/* --- model setup (host arrays are copied) ------------------------------ */
orc_model* orc_create(void);
void orc_destroy(orc_model* m);
const char* orc_last_error(const orc_model* m);
int orc_set_grid(orc_model* m, int nx, int ny, int nz, const double lo[3], const double hi[3]);
int orc_set_density(orc_model* m, const double* rho, size_t n);
int orc_set_frequencies(orc_model* m, const double* nu_edges, int n_nu);
int orc_set_dust(orc_model* m, const double* chi, const double* albedo, const double* g, int n_nu);
int orc_add_point_source(orc_model* m, const double pos[3], double lum, double teff);
int orc_add_point_source_spectrum(orc_model* m, const double pos[3], double lum,
                                  const double* l_nu_bin, int n_nu);
int orc_set_observers(orc_model* m, int n_incl, int img_npix, double img_half_width,
                      const int* img_nu_bins, int n_img_nu);
int orc_set_run(orc_model* m, const orc_run_cfg* cfg);
int orc_set_temperature(orc_model* m, const double* T, size_t n);

/* --- running ------------------------------------------------------------ */
int orc_iterate(orc_model* m, orc_iter_stats* st);      /* one Lucy iteration */
int orc_final_pass(orc_model* m, orc_iter_stats* st);   /* binning pass at fixed T */
/* Transport only: n packets with the iteration key of the next iteration,
 * accumulating into the model's absorption and binning arrays; used to time
 * the propagation on a bounded sample.  No temperature update. */
int orc_transport_sample(orc_model* m, int64_t n_packets, orc_iter_stats* st);
/* Packets [p_first, p_first+p_count) of a pass of np_total packets (energy
 * per packet L/np_total), the Lucy-iteration key of the next iteration or the
 * final-pass key; the event log covers packets from p_first on.  No
 * temperature update. */
int orc_transport_range(orc_model* m, int64_t np_total, int64_t p_first, int64_t p_count,
                        int final_pass, orc_iter_stats* st);

/* --- results ------------------------------------------------------------ */
int orc_get_specific_energy(const orc_model* m, double* adot, double* adot_sigma, size_t n);
int orc_get_temperature(const orc_model* m, double* T, size_t n);
int orc_get_absorbed_sum(const orc_model* m, double* acc, size_t n);  /* raw sum l*kappa */
/* raw sum of (l*kappa)^2 over the segments (kept only with want_noise) */
int orc_get_absorbed_sum2(const orc_model* m, double* acc2, size_t n);
int orc_get_sed(const orc_model* m, double* sum, double* sum2, int64_t* count, size_t n);
int orc_get_images(const orc_model* m, double* sum, double* sum2, size_t n);
/* Peeling-off (Sec. 2.6.2) toward n unit directions, in the final pass (and in
 * iterations with bin_every_iteration): SED [n][2][nnu] per steradian,
 * component 0 direct source emission, 1 scattered or re-emitted; images
 * [n_img][n][npix][npix] at the image bins of orc_set_observers. */
int orc_set_peeloff(orc_model* m, const double* dirs, int n);
int orc_get_peeled_sed(const orc_model* m, double* sum, double* sum2, size_t n);
int orc_get_peeled_images(const orc_model* m, double* sum, double* sum2, size_t n);
/* Raytracing (Sec. 2.6.3) of the dust's thermal emission at the current
 * temperatures and of the point sources toward the peel-off observers:
 * cube [n_peel][npix][npix][nnu] (erg/s/sr per pixel of an image over +-hw cm
 * on the peeled images' axes), sed [n_peel][2][nnu] (0 sources, 1 dust). */
int orc_raytrace(orc_model* m, int npix, double hw, double* cube, double* sed);
int orc_get_event_log(const orc_model* m, orc_event* ev, size_t cap, int32_t* counts, size_t n_counts);
int orc_get_emission_rows(const orc_model* m, int32_t* row, double* w, size_t n);

/* --- building blocks exposed for closed-form pins ----------------------- */
/* Modified random walk: y with F(y) = u for the escape-time distribution of
 * diffusion from the centre of a sphere, F(y) = 1 + 2 sum_n (-1)^n exp(-n^2 y)
 * (y = pi^2 D t / R^2), and F itself. */
double orc_mrw_escape_y(double u);
double orc_mrw_escape_cdf(double y);
/* Planck-mean absorption and Rosseland-mean extinction opacities of the
 * model's dust at temperature T over its bins (cm^2/g). */
double orc_planck_mean_kappa(const orc_model* m, double T);
double orc_rosseland_chi(const orc_model* m, double T);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* n-th FP64 uniform of the stream (key, packet). */
double orc_uniform(uint32_t key0, uint32_t key1, uint64_t packet, uint64_t n);
/* out[p*n_draws + n] = n-th uniform of packet packet0+p */
void orc_uniform_block(uint32_t key0, uint32_t key1, uint64_t packet0, int64_t n_packets,
                       int64_t n_draws, double* out);
/* isotropic unit vector from two uniforms (mu = 2u-1, phi = 2 pi u) */
void orc_isotropic(double u_mu, double u_phi, double d[3]);
/* integral of x^3/(e^x-1) over [a, b]; b may be +inf */
double orc_planck_x_integral(double a, double b);
/* integral of B_nu(T) over [nu_lo, nu_hi], erg s^-1 cm^-2 sr^-1 */
double orc_planck_bin(double nu_lo, double nu_hi, double T);
/* 4 pi sum_k kappa_k B_k(T) for the model's dust */
double orc_adot_of_T(const orc_model* m, double T);
/* T solving 4 pi sum_k kappa_k B_k(T) = adot; returns 1 K .. 1e4 K */
double orc_solve_T(const orc_model* m, double adot, int* clamped);
double orc_hg_mu(double g, double u);
void orc_rotate(const double d[3], double mu, double phi, double out[3]);
/* Walk a straight ray from x0 (inside the grid) along unit d until it leaves
 * the grid; writes up to cap (cell index, segment length) pairs; returns the
 * number of segments, or -1 if cap is too small. */
int64_t orc_trace_ray(const orc_model* m, const double x0[3], const double d[3],
                      int64_t* cells, double* lengths, int64_t cap);
/* nearest-rank percentile: the ceil(p*n)-th smallest value (1-based) */
double orc_percentile(const double* v, int64_t n, double p);

#ifdef __cplusplus
}
#endif
#endif
