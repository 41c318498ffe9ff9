/*
 * mcrt.h -- C ABI of the MI355X Monte-Carlo dust continuum radiative transfer
 * library (libmcrt.so).  The method is that of Robitaille (2011), HYPERION:
 * photon packets emitted by point sources propagate through a 3-D Cartesian
 * grid of constant-density cells; at each interaction they scatter
 * (Henyey-Greenstein) or are absorbed and immediately re-emitted; the Lucy
 * path-length estimator gives the specific energy absorption rate of every
 * cell, from which the LTE temperature follows; the iteration repeats until
 * the absorbed energy has converged, and a final pass bins escaping packets
 * into SEDs and images.
 *
 * Conventions
 *   - cgs units: cm, g, s, erg, Hz, K.
 *   - Cell arrays are C-ordered with x fastest: j = i + nx*(jy + ny*k).
 *   - Frequency bins are ordered by increasing frequency; a packet carries a
 *     bin index (multigroup); dust properties are constant over a bin.
 *   - Host input arrays are copied during the call; device input pointers
 *     are read during the call only and never retained.
 *   - Output buffers are owned by the caller; their element count n is
 *     checked (MCRT_E_SIZE when it does not match).
 *   - The library owns every device allocation it makes and frees it in
 *     mcrt_destroy.  Nothing crosses the ABI as an exception, abort or print:
 *     functions return a status and keep a per-model message.
 *   - Threading: one model per host thread; models are independent.
 *   - Every numerical step runs in HIP kernels on the model's device; the
 *     host only validates, builds FP64 tables once and schedules launches.
 */
#ifndef MCRT_H
#define MCRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mcrt_model mcrt_model;

typedef enum {
    MCRT_OK = 0,
    MCRT_E_ARG = -1,         /* invalid argument value                        */
    MCRT_E_STATE = -2,       /* call out of order (e.g. iterate before setup) */
    MCRT_E_NOMEM = -3,       /* device or host allocation failed              */
    MCRT_E_DEVICE = -4,      /* a HIP call failed                             */
    MCRT_E_UNSUPPORTED = -5, /* option not available                          */
    MCRT_E_SIZE = -6         /* caller buffer size does not match             */
} mcrt_status;

typedef enum {
    MCRT_FP64 = 0,           /* FP64 transport: same-stream parity path        */
    MCRT_FP32_TRANSPORT = 1  /* FP32 packet transport, FP64 reductions/tables  */
} mcrt_precision;

/* Event types of the per-packet log. */
enum { MCRT_EV_EMIT = 0, MCRT_EV_SCATTER = 1, MCRT_EV_ABSORB = 2, MCRT_EV_ESCAPE = 3,
       MCRT_EV_KILLED = 4, MCRT_EV_MRW = 5 };

/* One event.  cell: the cell of the event (for ESCAPE the last cell inside the
 * grid); nu: frequency bin after the event; incl: SED inclination bin of an
 * ESCAPE, else -1. */
typedef struct {
    int64_t packet;
    int32_t index;
    int32_t type;
    int32_t cell[3];
    int32_t nu;
    int32_t incl;
    int32_t reserved;
} mcrt_event;

/* Run parameters (mcrt_run_cfg_default fills the defaults in brackets). */
typedef struct {
    int64_t n_packets;         /* source packets per Lucy iteration [1e5] (Sec. 2.2)      */
    int64_t n_packets_final;   /* packets of the final binning pass [= n_packets]         */
    int32_t n_iter;            /* maximum Lucy iterations of mcrt_run [5]                 */
    int32_t precision;         /* mcrt_precision [MCRT_FP64]                              */
    uint64_t seed;             /* Philox key word 0 = seed mod 2^32 [1]                   */
    double t_init;             /* initial temperature, K [10]                             */
    int64_t max_events;        /* interactions before a packet is killed [1e6]            */
    double conv_p;             /* percentile p of Sec. 2.4 [0.999]                        */
    double conv_q_thres;       /* Q_thres [2]                                             */
    double conv_d_thres;       /* Delta_thres [1.1]                                       */
    double conv_dT_thres;      /* max |dT/T| threshold [0.01]                             */
    double conv_noise_thres;   /* noise mask: sigma_dT/T limit when want_noise [0.002]    */
    int32_t stop_on_convergence; /* 0 none, 1 max dT/T, 2 Q/Delta [0]                     */
    int32_t source_sampling;   /* 0 luminosity-proportional, 1 equal numbers [0]          */
    int32_t want_noise;        /* also accumulate sum of squared weights [0]              */
    int32_t event_log_packets; /* log events of packets [0, this) of each pass [0]        */
    int32_t event_log_cap;     /* events kept per logged packet [256]                     */
    int32_t bin_every_iteration; /* bin escapes into SED/images in Lucy iterations too [0]*/
    int32_t block_size;        /* transport threads per block, multiple of 64, at most
                                  256 (768 for FP32 tiled sweeps, 512 when a pass logs,
                                  bins or walks modified random walks); 0: 768 (512) for
                                  FP32 tiled sweeps, else 256 [0]                         */
    int32_t blocks_per_cu;     /* persistent blocks per compute unit [0 = occupancy]      */
    int32_t defer_lanes;       /* lanes of a wave that wait before events run (tiled
                                  sweeps: interactions, escapes, exits and free lanes with
                                  a record to take); 0: 16 for the per-lane walk, 40 for
                                  tiled sweeps [0]                                        */
    int32_t walk_batch;        /* grid segments a lane gathers per walk step of the
                                  per-lane walk: 1,2,4,8 [4]; tiled sweeps walk 4         */
    int32_t grid_layout;       /* device layout of the transport grid: 0 x-fastest,
                                  1 bricks of 4x4x4 cells [0]; results are identical     */
    int32_t tally_copies;      /* absorption tallies per device: 1, or 8 (one per XCD,
                                  summed by the cell update) [8]                          */
    int32_t transport_mode;    /* 0: every lane walks its packet through the whole grid,
                                  tallies with global FP64 atomics; 1: tiled sweeps --
                                  packets grouped by tile of tile_xy^2 x tile_z cells, each
                                  tile walked with density and tally in LDS, tally flushed
                                  to FP64 when a workgroup leaves the tile [1]; same packet
                                  histories.  Tiled sweeps hold at most 1024 cells per
                                  axis (MCRT_E_UNSUPPORTED beyond).  The tiled sweeps win
                                  on grids where most cells hold dust and packets cross
                                  many of them (5-6x on 128^3-256^3 clumps); the per-lane
                                  walk on small or mostly empty grids (6.8x on a 32^3
                                  sphere, 1.7x on a 128^3 disk), where a tile's load and
                                  flush serve few records                                 */
    int32_t tile_z;            /* tiled sweeps: tile extent in z, 1..64, halved while the
                                  tile does not fit in LDS; 0: 20 in FP32, 32 in FP64 [0] */
    int32_t visit_events;      /* tiled sweeps: interactions per tile visit before a
                                  packet waits for the next sweep [256]                   */
    int32_t tile_xy;           /* tiled sweeps: tile extent in x and y, a multiple of 4 in
                                  [4, 64]; 0: 24 in FP32, 16 in FP64 [0].  A tile holds its
                                  density (transport precision) and its FP64 tally in LDS */
    double mrw_gamma;          /* modified random walk (Sec. 2.2): at the start of a flight,
                                  while the sphere to the nearest wall of the cell holds at
                                  least mrw_gamma Rosseland mean free paths, one diffusion
                                  step to its surface (path length from the first-passage
                                  distribution, tally with the Planck-mean absorption,
                                  re-emission from the cell); 0 = off [0]                 */
    int64_t sweep_batch;       /* tiled sweeps: packets emitted at a time; whenever fewer
                                  records than this are in flight after a sweep, the next
                                  sweep_batch packets are emitted into the pool (refill);
                                  0: as many as two record buffers (about 2.7 batches of
                                  80-byte FP32 or 144-byte FP64 records each) hold in 30 %
                                  of the device memory: 2e8 (FP32) or 1.1e8 (FP64) packets
                                  on a 288 GB MI355X, at least 2^25 [0]                   */
    int64_t sweep_drain;       /* tiled sweeps: once every packet is emitted and at most
                                  this many records remain, the per-lane walk finishes
                                  them in one launch instead of further sweeps (same
                                  histories); 0: the smaller of 2^18 and 1/64 of the
                                  pass's packets, -1: never [0]                           */
} mcrt_run_cfg;

/* Statistics of one pass (a Lucy iteration or the final pass). */
typedef struct {
    int32_t iteration;         /* index of the iteration just finished                    */
    int32_t converged_q;       /* Q < Q_thres and Delta < Delta_thres (Eqs. 4-6)          */
    int32_t converged_dT;      /* max over the mask of |dT/T| < conv_dT_thres             */
    int32_t precision;
    double q;                  /* p-th percentile of R_j (Eq. 5); +inf without history    */
    double delta;              /* delta(Q^{i-1}, Q^i) (Eq. 6)                             */
    double max_dT;             /* max over the mask of |T^i - T^{i-1}| / T^{i-1}          */
    double p999_dT;            /* 99.9th percentile of the same                           */
    int64_t n_mask;            /* cells in the dT mask                                    */
    int64_t n_r;               /* cells entering the percentile of R                      */
    int64_t n_unsampled;       /* dust cells with zero absorption (T set to 1 K)          */
    int64_t n_t_clamped;       /* cells whose T was clamped to [1 K, 1e4 K]               */
    int64_t n_row_clamped;     /* dust cells whose emission row was clamped               */
    int64_t n_cross_dust;      /* walk segments in cells with rho > 0                     */
    int64_t n_cross_empty;     /* walk segments in cells with rho = 0                     */
    int64_t n_scatter;
    int64_t n_absorb;
    int64_t n_escape;
    int64_t n_killed;
    double e_escaped;          /* energy of escaped packets, erg (Delta t = 1 s)          */
    double e_killed;           /* energy of killed packets, erg                           */
    double ms_transport;       /* device time of the transport kernel(s)                  */
    double ms_update;          /* device time of the temperature update and statistics    */
    double ms_total;           /* host wall time of the call                              */
    int64_t n_sweeps;          /* tiled sweeps run by the pass (transport_mode 1)         */
    int64_t n_visits;          /* tile visits (packet records walked) over those sweeps   */
    int64_t n_mrw;             /* modified-random-walk steps                              */
    double ms_dominant;        /* device time of the pass's dominant kernel, summed over
                                  its launches (tiled sweeps: every sweep kernel and the
                                  per-lane finish of the tail; per-lane walk: the one
                                  transport launch)                                       */
    int64_t n_drained;         /* tiled sweeps: records of the tail finished per lane     */
} mcrt_iter_stats;

typedef struct {
    int32_t n_iterations;      /* Lucy iterations run                                     */
    int32_t converged;         /* the stopping criterion was met                          */
    int32_t first_converged;   /* first iteration meeting the criterion, -1 if none       */
    int32_t reserved;
    double ms_total;           /* wall time of mcrt_run                                   */
    double ms_to_converged;    /* wall time until the end of first_converged              */
    mcrt_iter_stats last;      /* statistics of the last Lucy iteration                   */
    mcrt_iter_stats final_pass;
} mcrt_run_stats;

/* ---- lifetime ------------------------------------------------------------ */
/* A model holds one problem of Sec. 2.1 (grid, density, dust, sources) and its
 * state on HIP device hip_device.  *out receives the handle (NULL on failure:
 * MCRT_E_DEVICE for a bad device, MCRT_E_NOMEM).  Plumbing, not a passage of
 * the paper. */
mcrt_status mcrt_create(mcrt_model** out, int hip_device);
/* Frees every device and host allocation of m.  NULL-safe. */
void mcrt_destroy(mcrt_model* m);
/* Message of the last failing call on m; valid until the next call on m. */
const char* mcrt_last_error(const mcrt_model* m);
/* Run all work of m on this HIP stream (e.g. a PyTorch stream handle); NULL =
 * the library's own stream.  The stream must outlive the model's use of it. */
mcrt_status mcrt_set_stream(mcrt_model* m, void* hip_stream);

/* ---- problem (Sec. 2.1) -------------------------------------------------- */
/* Cartesian grid of nx*ny*nz cells over [lo, hi] (Sec. 2.1.2). */
mcrt_status mcrt_set_grid(mcrt_model* m, int nx, int ny, int nz, const double lo[3],
                          const double hi[3]);
/* Dust density per cell (Sec. 2.1.2: cells of constant density), g cm^-3,
 * finite and >= 0, host array of n = ncell values in the cell order above,
 * copied during the call.  MCRT_E_STATE before mcrt_set_grid, MCRT_E_SIZE for
 * another n, MCRT_E_ARG for a negative or non-finite value. */
mcrt_status mcrt_set_density(mcrt_model* m, const double* rho, size_t n);
/* Same from device memory (FP64 if is_fp64 else FP32), read during the call
 * (Sec. 2.1.2). */
mcrt_status mcrt_set_density_device(mcrt_model* m, const void* d_rho, int is_fp64, size_t n);
/* n_nu+1 strictly increasing frequency edges, Hz (host array, copied).  The
 * bins carry the source spectra (Sec. 2.1.1) and the dust properties
 * (Sec. 2.1.3): a packet keeps the index of its bin.  MCRT_E_ARG for edges
 * that are not positive and increasing. */
mcrt_status mcrt_set_frequencies(mcrt_model* m, const double* nu_edges, int n_nu);
/* Mass extinction chi_nu (cm^2/g, >= 0), albedo in [0,1] and HG asymmetry g,
 * |g| < 1, per bin (Sec. 2.1.3).  kappa = chi (1 - albedo). */
mcrt_status mcrt_set_dust(mcrt_model* m, const double* chi, const double* albedo, const double* g,
                          int n_nu);
/* Isotropic point source with a blackbody spectrum of teff (Sec. 2.1.1); the
 * spectrum is truncated to the bins and renormalised to lum (erg/s). */
mcrt_status mcrt_add_point_source(mcrt_model* m, const double pos[3], double lum, double teff);
/* Isotropic point source with a given relative luminosity per bin. */
mcrt_status mcrt_add_point_source_spectrum(mcrt_model* m, const double pos[3], double lum,
                                           const double* l_nu_bin, int n_nu);
/* SED and image binning of escaping packets (Sec. 2.6.1): n_incl bins of
 * |d_z|; images of img_npix^2 pixels over +-img_half_width (cm) for the listed
 * frequency bins. */
mcrt_status mcrt_set_observers(mcrt_model* m, int n_incl, int img_npix, double img_half_width,
                               const int* img_nu_bins, int n_img_nu);
/* Peeling-off (Sec. 2.6.2) toward n observers (unit vectors dirs[3*i..3*i+2]):
 * at each source emission, scattering and re-emission of a binning pass (the
 * final pass, or every iteration with bin_every_iteration), a packet of weight
 * eps p exp(-tau) is added toward every observer, p the probability per
 * steradian of leaving in that direction (1/(4 pi) for emission and
 * re-emission, the Henyey-Greenstein phase function for scattering) and tau
 * the optical depth from the event to the grid boundary in the packet's bin.
 * Call after mcrt_set_observers; images use its image bins, pixels and width. */
mcrt_status mcrt_set_peeloff(mcrt_model* m, const double* dirs, int n);
/* Peeled SED [n][2][n_nu] (erg/s per sr; component 0 direct source light,
 * 1 scattered or re-emitted): sums and sums of squares of the peeled weights. */
mcrt_status mcrt_get_peeled_sed(mcrt_model* m, double* sum, double* sum2, size_t n);
/* Peeled images [n_img][n][npix][npix]: e_x = norm(z x o), e_y = o x e_x. */
mcrt_status mcrt_get_peeled_images(mcrt_model* m, double* sum, double* sum2, size_t n);
/* Raytracing (Sec. 2.6.3) of the emission toward the peel-off observers, in
 * post-processing at the current temperatures.  Per observer o an image of
 * npix x npix pixels over +-half_width (cm) around the grid centre on the axes
 * of the peeled images; through each pixel centre one ray, followed from the
 * observer's side of the grid along -o, sums in every frequency bin k the
 * formal solution through cells of constant density and temperature:
 *     I_k = sum over cells, front to back, exp(-tau_k in front) S_k (1 - exp(-dtau_k)),
 * dtau_k = rho chi_k l (l the chord), S_k = (kappa_k / chi_k) B_k(T): the
 * dust's thermal emission over extinction, B_k the bin-integrated Planck
 * function per sr.  Scattered light is not included (that is peeling-off's
 * share).  Pixel values are I_k times the pixel area (erg/s/sr); each point
 * source adds L_k/(4 pi) exp(-tau_k(source -> boundary along o)) to the pixel
 * it projects into.  The SED is the pixel sum, so half_width should cover the
 * grid; it is a quadrature of the image plane that needs pixels small against
 * the cells' projection.  Needs mcrt_set_peeloff; the model keeps the cube
 * (n_peel*npix^2*n_nu doubles, at most 2^34) until the next call or destroy. */
mcrt_status mcrt_raytrace(mcrt_model* m, int npix, double half_width);
/* Partial diffusion approximation (Appendix A) after a Lucy iteration: dust
 * cells whose absorption estimate is zero, or (with want_noise) whose relative
 * error exceeds noise, take T from div(D grad T^4) = 0, D = 1/(3 rho chi_R),
 * with the other dust cells as boundary values.  Cartesian form of the
 * appendix's discrete equation: a face between cells c and n (axis a) has the
 * conductance 1/(dx_a^2 (rho_c chi_R,c + rho_n chi_R,n)); empty cells and the
 * outside carry no flux; chi_R is the Rosseland mean at the current T, the
 * linear system is solved passes times (Picard) by conjugate gradients to a
 * relative residual of 1e-12.  Groups of such cells with no other dust cell
 * next to them keep their T.  Sets T, Adot (Eq. 3) and the emission of the
 * solved cells for the next iteration. */
typedef struct {
    int64_t n_pda;             /* cells selected                                          */
    int64_t n_solved;          /* of them connected to a sampled cell, given a new T      */
    int32_t passes;            /* linear solves done                                      */
    int32_t cg_iterations;     /* conjugate-gradient iterations of the last solve         */
    double residual;           /* its relative residual |b - A x| / |b|                   */
} mcrt_pda_stats;
mcrt_status mcrt_apply_pda(mcrt_model* m, double noise, int passes, mcrt_pda_stats* st);
/* Raytraced SED [n_peel][2][n_nu] (erg/s/sr): 0 point sources, 1 dust. */
mcrt_status mcrt_get_raytraced_sed(mcrt_model* m, double* sed, size_t n);
/* Raytraced spectral cube [n_peel][npix][npix][n_nu] (erg/s/sr per pixel,
 * dust and sources), host copy or the device pointer (valid until the next
 * mcrt_raytrace or mcrt_destroy). */
mcrt_status mcrt_get_raytraced_cube(mcrt_model* m, double* cube, size_t n);
mcrt_status mcrt_get_raytraced_cube_device(mcrt_model* m, const double** d_cube);
/* Fill cfg with the defaults in brackets above. */
mcrt_status mcrt_run_cfg_default(mcrt_run_cfg* cfg);
/* Photon counts, iterations and convergence thresholds (Sec. 2.2, 2.4) and
 * launch options; copied.  MCRT_E_ARG for an out-of-range field. */
mcrt_status mcrt_set_run(mcrt_model* m, const mcrt_run_cfg* cfg);
/* Temperatures (K, > 0; n = ncell, host, copied) that the next Lucy iteration
 * re-emits from (Sec. 2.3-2.4: the emissivity of an iteration follows from the
 * previous one's absorption rate; here from T, the start of the iteration). */
mcrt_status mcrt_set_temperature(mcrt_model* m, const double* T, size_t n);
/* Same from device memory (FP64 if is_fp64 else FP32), read during the call. */
mcrt_status mcrt_set_temperature_device(mcrt_model* m, const void* d_T, int is_fp64, size_t n);

/* ---- running ------------------------------------------------------------- */
/* One Lucy iteration (Sec. 2.3-2.4): transport n_packets with the emission of
 * the current temperatures, Ȧ by Eq. 2, T by Eq. 3, convergence statistics. */
mcrt_status mcrt_iterate(mcrt_model* m, mcrt_iter_stats* st);
/* Final binning pass at fixed temperatures (Sec. 2.6.1); Ȧ is not updated. */
mcrt_status mcrt_final_pass(mcrt_model* m, mcrt_iter_stats* st);
/* Lucy iterations (Sec. 2.3) until n_iter or the stopping criterion of
 * Sec. 2.4 (Eqs. 4-6, or max dT/T), then the final binning pass (Sec. 2.6.1). */
mcrt_status mcrt_run(mcrt_model* m, mcrt_run_stats* st);

/* ---- results ------------------------------------------------------------- */
/* Specific energy absorption rate of every cell after the last Lucy
 * iteration, Eq. 2: Adot = eps sum(l kappa) / (dt V), dt = 1 s, erg/s/g;
 * adot_sigma (may be NULL) its Monte-Carlo standard error from the sum of
 * squared path-length weights (needs want_noise, else zeros).  n = ncell. */
mcrt_status mcrt_get_specific_energy(mcrt_model* m, double* adot, double* adot_sigma, size_t n);
/* LTE temperature of every cell, K: the root of 4 pi sum_k kappa_k B_k(T) = Adot
 * (Eq. 3 over the model's bins); dust cells with Adot = 0 hold 1 K.  n = ncell. */
mcrt_status mcrt_get_temperature(mcrt_model* m, double* T, size_t n);
/* Device pointer to the FP64 temperature field (valid until the next call). */
mcrt_status mcrt_get_temperature_device(mcrt_model* m, const double** d_T);
/* Binned SED of the last binning pass (Sec. 2.6.1; uncertainties from the
 * sums of squares, Sec. 2.7.1) [n_incl][n_nu]: sum of escaped energies (erg,
 * dt = 1 s), sum of their squares, packet counts; n = n_incl*n_nu. */
mcrt_status mcrt_get_sed(mcrt_model* m, double* sum, double* sum2, int64_t* count, size_t n);
/* Binned images (Sec. 2.6.1) [n_img_nu][n_incl][npix][npix]: the escape point
 * projected on e_x = norm(z x d), e_y = d x e_x (row index from Y, column from
 * X); sum of energies and of squares. */
mcrt_status mcrt_get_images(mcrt_model* m, double* sum, double* sum2, size_t n);
/* Event log of the last pass (the packet history of Sec. 2.2: emission,
 * scatterings, absorptions, escape): ev[p*cap + i], counts[p] events of
 * packet p (may exceed cap: later events were dropped).  Returns MCRT_OK. */
mcrt_status mcrt_get_event_log(mcrt_model* m, mcrt_event* ev, size_t cap_total, int32_t* counts,
                               size_t n_counts);
/* The direction update of a scattering (Sec. 2.2 with the Henyey-Greenstein
 * phase function): for i < n, out[3i..3i+2] = the unit vector at angle acos(mu[i])
 * from the unit vector d[3i..3i+2], azimuth phi[i] about it, computed on m's
 * device by the device function every transport kernel uses, in precision
 * MCRT_FP64 or MCRT_FP32_TRANSPORT (inputs rounded to FP32 first).  Host
 * arrays, copied; MCRT_E_ARG for mu outside [-1, 1] or non-finite values. */
mcrt_status mcrt_scatter_directions(mcrt_model* m, int precision, const double* d, const double* mu,
                                    const double* phi, double* out, int n);
/* The same directions as mcrt_scatter_directions, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): this call allocates nothing.  Its device
 * staging is a static array of at most 65536 directions (9 doubles each) that
 * each GPU holds for the life of the process; n above that gives MCRT_E_SIZE.
 * All calls on one GPU share that array: calls that overlap on a GPU (other
 * host threads, other streams) race and must be serialised by the caller. */
mcrt_status mcrt_scatter_directions_noalloc(mcrt_model* m, int precision, const double* d, const double* mu,
                                            const double* phi, double* out, int n);
/* Number of compute units and the wavefront width of the model's device
 * (plumbing, not a passage of the paper). */
mcrt_status mcrt_device_info(mcrt_model* m, int* n_cu, int* wave_size);

/* ---- batching: many independent models in one launch ---------------------
 * Sec. 3 of the paper: packets are independent within an iteration, so the
 * packets of many small models can share one persistent launch.  Each model
 * keeps its own grid, dust, sources, seed, packet count and results; a model's
 * results equal those of its own mcrt_iterate calls up to the order of FP64
 * summation.  Per-model percentile statistics (q, p999_dT) are not computed
 * in batches. */
typedef struct {
    int32_t n_iter;            /* Lucy iterations [5]                                      */
    int32_t final_pass;        /* then the final binning pass [1]                          */
    int32_t use_graph;         /* replay iterations after the first from a hipGraph [1]    */
    int32_t autotune;          /* choose the launch shape by timing calibration runs [1]   */
    int32_t block_size;        /* threads per block; 0 = tuned or 256                      */
    int32_t walk_batch;        /* 0 = tuned or 4                                           */
    int32_t defer_lanes;       /* 0 = tuned or 16                                          */
    int32_t blocks_per_cu;     /* 0 = tuned or occupancy limit                             */
    double tune_fraction;      /* packet fraction of each calibration run [0.02]           */
    int32_t verbose;           /* 1: a line on stderr after each iteration [0]             */
} mcrt_batch_cfg;

typedef struct {
    int32_t n_models;
    int32_t n_iterations;
    int32_t graph_used;
    int32_t tuned;             /* 1 measured now, 2 from the tuning cache, 0 not tuned     */
    int32_t block_size, walk_batch, defer_lanes, blocks_per_cu;  /* launch shape used      */
    int64_t packets_per_iteration;
    int64_t n_cross_dust;      /* summed over models, last iteration                       */
    int64_t n_cross_empty;
    double ms_total;           /* wall time of the call                                    */
    double ms_iterations;      /* wall time of the Lucy iterations                         */
    double ms_final;           /* wall time of the final pass                              */
    double ms_tune;            /* wall time of autotuning                                  */
    double ms_transport_last;  /* device time of the last batched transport launch         */
} mcrt_batch_stats;

mcrt_status mcrt_batch_cfg_default(mcrt_batch_cfg* cfg);
/* All models: same device and precision, fully set up.  The work runs on the
 * first model's stream.  Returns the first failing model's status; the error
 * message is then on models[0]. */
mcrt_status mcrt_batch_run(mcrt_model* const* models, int n, const mcrt_batch_cfg* cfg,
                           mcrt_batch_stats* st);

/* ---- learned warm start --------------------------------------------------
 * The Lucy iteration (Sec. 2.4) converges from any starting temperature; its
 * cost is the number of iterations.  A 3-D convolutional encoder-decoder
 * predicts log10 T per cell from two features of the problem and is used as
 * the starting temperature; Monte-Carlo iterations then decide convergence
 * exactly as from a cold start.
 *
 * Network: 4 levels of C, 2C, 4C, 8C channels (C = base_channels, 16 or 32),
 * two 3x3x3 convolutions (zero padding) per level, 2x2x2 stride-2 down
 * convolutions and transposed up convolutions, skip concatenation [up, skip]
 * in the decoder, LeakyReLU(0.1) after every convolution, a 1x1x1 head.  BF16
 * weights and activations on the matrix cores with FP32 accumulation; FP32
 * master parameters trained with Adam (b1 0.9, b2 0.999, eps 1e-8).
 *
 * Tensors of a batch are N cubes of side D (D a multiple of 8), voxel index
 * ((n*D + z)*D + y)*D + x.  Features x: FP32 [N][D^3][3] (see
 * mcrt_model_features); outputs y: FP32 [N][D^3], log10 T in K.
 * Parameter vector (FP32): per layer in network order, weights
 * [taps][C_out][C_in] (taps 27 = dz*9 + dy*3 + dx for 3x3x3 with offsets
 * -1..1, 8 = tz*4 + ty*2 + tx for 2x2x2) then biases [C_out]; the head's
 * weights [C] and bias last.  The first layer sees the features scaled as
 * (x0 + 2)/2, (x1 + 30)/10, (x2 - 4)/3 in input channels 0-2; its input
 * channels 3..15 see zeros.  Device pointers are in the surrogate's device memory; the calls
 * synchronise the surrogate's stream before returning. */
typedef struct mcrt_surrogate mcrt_surrogate;

mcrt_status mcrt_surrogate_create(mcrt_surrogate** out, int hip_device, int base_channels,
                                  uint64_t seed);           /* He-normal init from seed */
void mcrt_surrogate_destroy(mcrt_surrogate* s);            /* NULL-safe                */
const char* mcrt_surrogate_last_error(const mcrt_surrogate* s);
mcrt_status mcrt_surrogate_set_stream(mcrt_surrogate* s, void* hip_stream);
int64_t mcrt_surrogate_param_count(const mcrt_surrogate* s);
/* Host copies of the FP32 parameters / of the gradients of the last train step.
 * Saving and loading a trained network is host file I/O over these two calls
 * (the Python binding writes the parameter vector as a .npy file); the
 * library itself reads and writes no files. */
mcrt_status mcrt_surrogate_get_params(mcrt_surrogate* s, float* host, size_t n);
mcrt_status mcrt_surrogate_set_params(mcrt_surrogate* s, const float* host, size_t n);
mcrt_status mcrt_surrogate_get_grads(mcrt_surrogate* s, float* host, size_t n);
/* Inference: d_y[v] = log10 T predicted for voxel v. */
mcrt_status mcrt_surrogate_forward(mcrt_surrogate* s, const float* d_x, int N, int D, float* d_y);
/* One training step on a batch: loss = sum_v mask_v (y_v - target_v)^2 /
 * mask_count (mask 0 or 1 per voxel, FP32), its gradient with respect to all
 * parameters, then (apply_update != 0) one Adam step with learning rate lr.
 * *loss receives the loss before the update. */
mcrt_status mcrt_surrogate_train_step(mcrt_surrogate* s, const float* d_x, const float* d_target,
                                      const float* d_mask, int N, int D, double mask_count,
                                      double lr, int apply_update, double* loss);
/* Scale the gradient of later train steps by min(1, max_norm / ||g||_2) before
 * the Adam update (0, the default, turns clipping off). */
mcrt_status mcrt_surrogate_set_grad_clip(mcrt_surrogate* s, double max_norm);
/* Inference written as temperatures: d_T[v] = 10^y clamped to [1, 1e4] K (FP64). */
mcrt_status mcrt_surrogate_predict_T(mcrt_surrogate* s, const float* d_x, int N, int D, double* d_T);

/* Features of a model for the network, FP32 [ncell][3] in device memory
 * (n = 3*ncell), from the density, the dust and the sources:
 *   0: log10 max(rho chi(1 um) dx, 1e-6), the optical depth of one cell width
 *      at 1 micron (chi of the bin holding 1 um, dx the x cell width);
 *   1: log10(D + 1e-30), the deposit field D = (sum of the luminosities of the
 *      sources in the cell) / (4 pi dx^2) in erg s^-1 cm^-2, a source on a cell
 *      wall, edge or corner being shared equally by the cells that touch it;
 *   2: log10(sum over deposit cells c of D_c dx^2 / max(r^2, dx^2/4) + 1e-30),
 *      r the distance between cell centres: the deposit field spread by the
 *      free-space 1/r^2 kernel (the unattenuated flux of the deposited light). */
mcrt_status mcrt_model_features(mcrt_model* m, float* d_x, size_t n);
/* Warm start: features -> network -> temperatures of m (as by
 * mcrt_set_temperature_device).  The grid must be a cube of cells with a side
 * that is a multiple of 8.  *ms (may be NULL) receives the wall time. */
mcrt_status mcrt_warm_start(mcrt_model* m, mcrt_surrogate* s, double* ms);

#ifdef __cplusplus
}
#endif
#endif /* MCRT_H */
