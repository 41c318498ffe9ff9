/*
 * orc.c -- plain FP64 CPU oracle for Monte-Carlo dust continuum radiative
 * transfer, written from Robitaille (2011), "HYPERION: an open-source
 * parallelized three-dimensional dust continuum radiative transfer code".
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  It shares no
 * code with the HIP library.  Slow and direct on purpose: one packet at a
 * time, scalar FP64, no blocking or fusion.
 *
 * What it follows (paper sections / equations):
 *   Sec. 2.1.1  point sources with a luminosity and a spectrum; isotropic.
 *   Sec. 2.1.3  dust given by chi_nu (mass extinction) and albedo; the
 *               scattering phase function is Henyey-Greenstein here (the
 *               paper uses a Mueller matrix; polarisation is not modelled).
 *               LTE emissivity j_nu = kappa_nu B_nu(T).
 *   Sec. 2.2    source selection by luminosity (or equal numbers with
 *               weights), tau = -ln(zeta), propagation until tau is reached
 *               or the packet escapes, absorb if zeta > albedo else scatter,
 *               repeat until escape.
 *   Sec. 1      immediate re-emission after absorption (energy conserved).
 *   Sec. 2.3    Eq. 2 (Lucy path-length estimator, Delta t = 1 s) and
 *               Eq. 3 (LTE balance; here over the model's frequency bins).
 *   Sec. 2.4    Eqs. 4-6 (delta, R_j, Q^i percentile, Delta^i).
 *   Sec. 3      the absorbed energy is frozen within an iteration; packets
 *               are independent, so chunked parallel work gives the same
 *               result up to summation order.
 *   Sec. 2.6.1  binning escaping packets into viewing-angle bins.
 *   Sec. 2.6.2  peeling-off: at each source emission, scattering and
 *               re-emission, weight p exp(-tau) toward each observer.
 *
 * Readings where the paper is silent (the same contract binds the HIP path):
 *   - multigroup frequencies: a packet carries a bin index; dust properties
 *     are constant over a bin; source spectra are truncated to the bins and
 *     renormalised so that the whole luminosity is carried;
 *   - emissivity rows: 128 rows log-spaced in T over [1 K, 1e4 K]; a cell
 *     re-emits from row m or m+1 chosen at random with the linear weight in
 *     log T of its temperature (unbiased for linear interpolation);
 *   - random numbers: Philox4x32-10 (Salmon et al. 2011), key = (seed mod
 *     2^32, iteration; final pass 0x80000000|iteration), counter = (call low,
 *     call high, packet low, packet high); one call gives two uniforms
 *     u = (floor(w/2^12) + 1/2) 2^-52 from the 64-bit words (x0:x1), (x2:x3);
 *   - draw order: emission u_src u_nu u_mu u_phi; each flight u_tau; each
 *     interaction u_int then (scatter) u_mu u_phi or (absorb) u_mix u_nu
 *     u_mu u_phi; every draw is consumed even when it cannot matter; a
 *     modified-random-walk step (mrw_gamma > 0, at the start of a flight)
 *     draws u_y u_mu u_phi u_mix u_nu u_mu u_phi;
 *   - grid walk: per axis the distance to the next wall; the smallest wins,
 *     ties go to the lowest axis (x, y, z) and one axis steps per segment;
 *     the stepped coordinate is set exactly onto the wall; walls are at
 *     lo + c*dx with dx = (hi-lo)/n; negative distances from rounding are
 *     taken as zero;
 *   - start cell: c = floor((x-lo)/dx) per axis, minus one when x sits
 *     exactly on that wall and the direction is negative on that axis;
 *   - cells whose absorption is zero get T = 1 K ("unsampled");
 *   - SED inclination bin = floor(n_incl*|d_z|) (folded over the mid-plane);
 *     images project the escape point on e_x = norm(z x d), e_y = d x e_x.
 *
 * Parity status: every building block is pinned by closed forms in the
 * tests (Philox known-answer vectors, Planck integrals against quadrature
 * and pi^4/15, HG and isotropic moments, grid walk against chord lengths
 * and brute force, slab transmission exp(-tau), luminosity conservation,
 * the optically thin temperature profile).  End-to-end temperature and SED
 * values beyond those properties have no printed worked example in the
 * paper: parity unpinned there.
 */
#include "orc.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* CODATA 2018 / IAU 2015, cgs */
#define ORC_H_PLANCK 6.62607015e-27
#define ORC_K_BOLTZ 1.380649e-16
#define ORC_C_LIGHT 2.99792458e10
#define ORC_PI 3.14159265358979323846

#define ORC_NROW 128
#define ORC_T_LO 1.0
#define ORC_T_HI 1.0e4
#define ORC_T_FLOOR 1.0

enum { EV_EMIT = 0, EV_SCATTER = 1, EV_ABSORB = 2, EV_ESCAPE = 3, EV_KILLED = 4, EV_MRW = 5 };

/* ======================================================================= */
/* Philox4x32-10, from the published description (Salmon, Moraes, Dror &   */
/* Shaw 2011): 10 rounds of two 32x32->64 multiplies with a Weyl key bump. */
/* ======================================================================= */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static double words_to_uniform(uint32_t hi, uint32_t lo)
{
    uint64_t w = ((uint64_t)hi << 32) | (uint64_t)lo;
    uint64_t k = w >> 12; /* 52 bits */
    return ((double)k + 0.5) * 0x1p-52;
}

double orc_uniform(uint32_t key0, uint32_t key1, uint64_t packet, uint64_t n)
{
    uint64_t call = n >> 1;
    uint32_t ctr[4] = {(uint32_t)call, (uint32_t)(call >> 32), (uint32_t)packet,
                       (uint32_t)(packet >> 32)};
    uint32_t key[2] = {key0, key1};
    uint32_t out[4];
    orc_philox4x32_10(ctr, key, out);
    if ((n & 1) == 0) return words_to_uniform(out[0], out[1]);
    return words_to_uniform(out[2], out[3]);
}

typedef struct {
    uint32_t key0, key1;
    uint64_t packet;
    uint64_t n;
} orc_stream;

static double draw(orc_stream* s)
{
    double u = orc_uniform(s->key0, s->key1, s->packet, s->n);
    s->n++;
    return u;
}

/* ======================================================================= */
/* Planck function integrals.                                              */
/*   int_a^b x^3/(e^x-1) dx = G(b) - G(a),  G(x) = int_0^x                 */
/* Small x: G from the Bernoulli expansion x/(e^x-1) = sum B_n x^n/n!.     */
/* Large x: Phi(x) = int_x^inf by the series of Widger & Woodall (1976),   */
/*   Phi(x) = sum_n e^{-nx} (x^3/n + 3x^2/n^2 + 6x/n^3 + 6/n^4).           */
/* ======================================================================= */
#define ORC_X_SWITCH 1.5

static double planck_G_small(double x)
{
    /* even Bernoulli numbers B_2 .. B_30 */
    static const double B[15] = {
        1.0 / 6.0, -1.0 / 30.0, 1.0 / 42.0, -1.0 / 30.0, 5.0 / 66.0,
        -691.0 / 2730.0, 7.0 / 6.0, -3617.0 / 510.0, 43867.0 / 798.0, -174611.0 / 330.0,
        854513.0 / 138.0, -236364091.0 / 2730.0, 8553103.0 / 6.0,
        -23749461029.0 / 870.0, 8615841276005.0 / 14322.0};
    double x3 = x * x * x;
    double sum = x3 / 3.0 - x3 * x / 8.0;
    double xp = x3;          /* x^(n+3) with n = 0 */
    double fact = 1.0;       /* n! */
    for (int i = 0; i < 15; ++i) {
        int n = 2 * (i + 1);
        xp *= x * x;
        fact *= (double)(n - 1) * (double)n;
        double term = B[i] * xp / ((double)(n + 3) * fact);
        sum += term;
        if (fabs(term) < 1e-18 * fabs(sum)) break;
    }
    return sum;
}

static double planck_Phi_large(double x)
{
    if (x > 745.0) return 0.0;
    double x2 = x * x, x3 = x2 * x;
    double sum = 0.0;
    for (int n = 1; n < 200; ++n) {
        double dn = (double)n;
        double e = exp(-dn * x);
        double term = e * (x3 / dn + 3.0 * x2 / (dn * dn) + 6.0 * x / (dn * dn * dn) +
                           6.0 / (dn * dn * dn * dn));
        sum += term;
        if (term < 1e-18 * sum) break;
    }
    return sum;
}

double orc_planck_x_integral(double a, double b)
{
    if (!(b > a)) return 0.0;
    if (a < 0.0) a = 0.0;
    if (b <= ORC_X_SWITCH) return planck_G_small(b) - planck_G_small(a);
    double hi_part = planck_Phi_large(a > ORC_X_SWITCH ? a : ORC_X_SWITCH) -
                     (isinf(b) ? 0.0 : planck_Phi_large(b));
    if (a >= ORC_X_SWITCH) return hi_part;
    return (planck_G_small(ORC_X_SWITCH) - planck_G_small(a)) + hi_part;
}

double orc_planck_bin(double nu_lo, double nu_hi, double T)
{
    if (!(T > 0.0)) return 0.0;
    double kT = ORC_K_BOLTZ * T;
    double a = ORC_H_PLANCK * nu_lo / kT;
    double b = ORC_H_PLANCK * nu_hi / kT;
    double pref = 2.0 * pow(kT, 4) / (pow(ORC_H_PLANCK, 3) * ORC_C_LIGHT * ORC_C_LIGHT);
    return pref * orc_planck_x_integral(a, b);
}

/* x^3/(e^x - 1) */
static double planck_f(double x)
{
    if (x <= 0.0) return 0.0;
    if (x > 700.0) return 0.0;
    return x * x * x / expm1(x);
}

/* ======================================================================= */
/* Model.                                                                  */
/* ======================================================================= */
struct orc_model {
    char err[256];
    int have_grid, have_rho, have_nu, have_dust, have_run, have_obs;
    int n[3];
    double lo[3], hi[3], dx[3], vol;
    int64_t ncell;
    double* rho;
    int nnu;
    double* nu;    /* nnu+1 edges */
    double *chi, *alb, *g, *kap;
    /* sources */
    int nsrc, cap_src;
    double* spos;  /* 3 per source */
    double* slum;
    double* sspec; /* nsrc*nnu, luminosity per bin (unnormalised) */
    double* scdf;  /* nsrc*nnu cumulative */
    double* lcdf;  /* nsrc cumulative luminosity */
    double ltot;
    /* observers */
    int n_incl, npix, n_img;
    double img_hw;
    int* img_bins;
    int* img_of_bin; /* nnu -> image index or -1 */
    /* run */
    orc_run_cfg cfg;
    /* emissivity rows */
    double* ecdf;  /* ORC_NROW * nnu */
    double trow[ORC_NROW];
    /* state */
    int iter;       /* iterations done */
    double* T;
    double* T_prev;
    double* sig_rel;      /* sigma_T/T of the last iteration (0 if unknown) */
    double* sig_rel_prev;
    unsigned char* T_valid; /* T came from the user/initial value or a sampled cell */
    double* adot;
    double* adot_prev;
    double* adot_sig;
    int have_adot_prev;
    double q_prev;
    double* acc;
    double* acc2;
    int32_t* row_m;
    double* row_w;
    double* mrw_kp;   /* per cell, modified random walk: Planck-mean kappa at T */
    double* mrw_chir; /* and Rosseland-mean chi at T (cm^2/g)                   */
    double* sed_sum;
    double* sed_sum2;
    int64_t* sed_n;
    double* img_sum;
    double* img_sum2;
    /* peeling-off (Sec. 2.6.2): n_peel observer directions; SED [n_peel][2][nnu]
     * (component 0: direct source emission, 1: scattered or re-emitted) and
     * images [n_img][n_peel][npix][npix], energy per steradian */
    int n_peel;
    double* peel_dir;
    double* psed_sum;
    double* psed_sum2;
    double* pimg_sum;
    double* pimg_sum2;
    orc_event* evlog;
    int32_t* evcount;
    int ev_packets, ev_cap;
    int64_t ev_first;
};

static int fail(orc_model* m, const char* msg)
{
    snprintf(m->err, sizeof m->err, "%s", msg);
    return -1;
}

orc_model* orc_create(void)
{
    orc_model* m = (orc_model*)calloc(1, sizeof(orc_model));
    if (!m) return NULL;
    m->cfg.n_packets = 100000;
    m->cfg.n_packets_final = 100000;
    m->cfg.n_iter = 5;
    m->cfg.seed = 1;
    m->cfg.t_init = 10.0;
    m->cfg.max_events = 1000000;
    m->cfg.conv_p = 0.999;
    m->cfg.conv_q_thres = 2.0;
    m->cfg.conv_d_thres = 1.1;
    m->cfg.conv_dT_thres = 0.01;
    m->cfg.event_log_cap = 256;
    m->q_prev = INFINITY;
    for (int i = 0; i < ORC_NROW; ++i)
        m->trow[i] = exp(log(ORC_T_LO) + (double)i * (log(ORC_T_HI) - log(ORC_T_LO)) / (ORC_NROW - 1));
    return m;
}

static void free_state(orc_model* m)
{
    free(m->T); free(m->T_prev); free(m->T_valid); free(m->sig_rel); free(m->sig_rel_prev);
    free(m->adot); free(m->adot_prev); free(m->adot_sig);
    free(m->acc); free(m->acc2); free(m->row_m); free(m->row_w); free(m->mrw_kp); free(m->mrw_chir);
    m->mrw_kp = m->mrw_chir = NULL;
    m->T = m->T_prev = m->sig_rel = m->sig_rel_prev = NULL;
    m->T_valid = NULL;
    m->adot = m->adot_prev = m->adot_sig = m->acc = m->acc2 = m->row_w = NULL;
    m->row_m = NULL;
}

void orc_destroy(orc_model* m)
{
    if (!m) return;
    free(m->rho); free(m->nu); free(m->chi); free(m->alb); free(m->g); free(m->kap);
    free(m->spos); free(m->slum); free(m->sspec); free(m->scdf); free(m->lcdf);
    free(m->img_bins); free(m->img_of_bin); free(m->ecdf);
    free_state(m);
    free(m->sed_sum); free(m->sed_sum2); free(m->sed_n); free(m->img_sum); free(m->img_sum2);
    free(m->peel_dir); free(m->psed_sum); free(m->psed_sum2); free(m->pimg_sum); free(m->pimg_sum2);
    free(m->evlog); free(m->evcount);
    free(m);
}

const char* orc_last_error(const orc_model* m) { return m ? m->err : "null model"; }

int orc_set_grid(orc_model* m, int nx, int ny, int nz, const double lo[3], const double hi[3])
{
    if (nx < 1 || ny < 1 || nz < 1) return fail(m, "grid dimensions must be >= 1");
    for (int a = 0; a < 3; ++a)
        if (!(hi[a] > lo[a]) || !isfinite(lo[a]) || !isfinite(hi[a]))
            return fail(m, "grid bounds must be finite with hi > lo");
    m->n[0] = nx; m->n[1] = ny; m->n[2] = nz;
    m->vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        m->lo[a] = lo[a];
        m->hi[a] = hi[a];
        m->dx[a] = (hi[a] - lo[a]) / (double)m->n[a];
        m->vol *= m->dx[a];
    }
    m->ncell = (int64_t)nx * ny * nz;
    free(m->rho); m->rho = NULL;
    free_state(m);
    m->have_grid = 1;
    m->have_rho = 0;
    m->iter = 0;
    return 0;
}

int orc_set_density(orc_model* m, const double* rho, size_t n)
{
    if (!m->have_grid) return fail(m, "set the grid first");
    if ((int64_t)n != m->ncell) return fail(m, "density size does not match the grid");
    for (size_t i = 0; i < n; ++i)
        if (!(rho[i] >= 0.0) || !isfinite(rho[i])) return fail(m, "density must be finite and >= 0");
    free(m->rho);
    m->rho = (double*)malloc(n * sizeof(double));
    memcpy(m->rho, rho, n * sizeof(double));
    m->have_rho = 1;
    return 0;
}

int orc_set_frequencies(orc_model* m, const double* nu_edges, int n_nu)
{
    if (n_nu < 1) return fail(m, "need at least one frequency bin");
    for (int k = 0; k <= n_nu; ++k)
        if (!(nu_edges[k] > 0.0) || !isfinite(nu_edges[k])) return fail(m, "frequency edges must be > 0");
    for (int k = 0; k < n_nu; ++k)
        if (!(nu_edges[k + 1] > nu_edges[k])) return fail(m, "frequency edges must increase");
    if (m->nsrc > 0) return fail(m, "set frequencies before adding sources");
    free(m->nu);
    m->nu = (double*)malloc((n_nu + 1) * sizeof(double));
    memcpy(m->nu, nu_edges, (n_nu + 1) * sizeof(double));
    m->nnu = n_nu;
    m->have_nu = 1;
    m->have_dust = 0;
    return 0;
}

static void build_emission_rows(orc_model* m);

int orc_set_dust(orc_model* m, const double* chi, const double* albedo, const double* g, int n_nu)
{
    if (!m->have_nu || n_nu != m->nnu) return fail(m, "dust size does not match the frequency bins");
    for (int k = 0; k < n_nu; ++k) {
        if (!(chi[k] >= 0.0) || !isfinite(chi[k])) return fail(m, "chi must be finite and >= 0");
        if (!(albedo[k] >= 0.0 && albedo[k] <= 1.0)) return fail(m, "albedo must be in [0,1]");
        if (!(fabs(g[k]) < 1.0)) return fail(m, "|g| must be < 1");
    }
    free(m->chi); free(m->alb); free(m->g); free(m->kap);
    m->chi = (double*)malloc(n_nu * sizeof(double));
    m->alb = (double*)malloc(n_nu * sizeof(double));
    m->g = (double*)malloc(n_nu * sizeof(double));
    m->kap = (double*)malloc(n_nu * sizeof(double));
    for (int k = 0; k < n_nu; ++k) {
        m->chi[k] = chi[k];
        m->alb[k] = albedo[k];
        m->g[k] = g[k];
        m->kap[k] = chi[k] * (1.0 - albedo[k]);
    }
    int any = 0;
    for (int k = 0; k < n_nu; ++k) any |= m->kap[k] > 0.0;
    if (!any) return fail(m, "dust must absorb in at least one bin");
    build_emission_rows(m);
    m->have_dust = 1;
    return 0;
}

/* Emissivity rows E[m][k]: cumulative distribution of kappa_k B_k(T_m). */
static void build_emission_rows(orc_model* m)
{
    free(m->ecdf);
    m->ecdf = (double*)malloc((size_t)ORC_NROW * m->nnu * sizeof(double));
    for (int r = 0; r < ORC_NROW; ++r) {
        double* row = m->ecdf + (size_t)r * m->nnu;
        double s = 0.0;
        for (int k = 0; k < m->nnu; ++k) {
            s += m->kap[k] * orc_planck_bin(m->nu[k], m->nu[k + 1], m->trow[r]);
            row[k] = s;
        }
        for (int k = 0; k < m->nnu; ++k) row[k] = s > 0.0 ? row[k] / s : (double)(k + 1) / m->nnu;
        row[m->nnu - 1] = 1.0;
    }
}

static int add_source(orc_model* m, const double pos[3], double lum, const double* lbin)
{
    if (!m->have_grid || !m->have_nu) return fail(m, "set grid and frequencies before sources");
    if (!(lum > 0.0) || !isfinite(lum)) return fail(m, "luminosity must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!(pos[a] >= m->lo[a] && pos[a] < m->hi[a])) return fail(m, "source outside the grid");
    double s = 0.0;
    for (int k = 0; k < m->nnu; ++k) {
        if (!(lbin[k] >= 0.0) || !isfinite(lbin[k])) return fail(m, "spectrum must be >= 0");
        s += lbin[k];
    }
    if (!(s > 0.0)) return fail(m, "spectrum has no power in the frequency bins");
    int i = m->nsrc;
    if (i == m->cap_src) {
        m->cap_src = m->cap_src ? 2 * m->cap_src : 8;
        m->spos = (double*)realloc(m->spos, 3 * m->cap_src * sizeof(double));
        m->slum = (double*)realloc(m->slum, m->cap_src * sizeof(double));
        m->sspec = (double*)realloc(m->sspec, (size_t)m->cap_src * m->nnu * sizeof(double));
        m->scdf = (double*)realloc(m->scdf, (size_t)m->cap_src * m->nnu * sizeof(double));
        m->lcdf = (double*)realloc(m->lcdf, m->cap_src * sizeof(double));
    }
    for (int a = 0; a < 3; ++a) m->spos[3 * i + a] = pos[a];
    m->slum[i] = lum;
    double c = 0.0;
    for (int k = 0; k < m->nnu; ++k) {
        m->sspec[(size_t)i * m->nnu + k] = lbin[k];
        c += lbin[k];
        m->scdf[(size_t)i * m->nnu + k] = c / s;
    }
    m->scdf[(size_t)i * m->nnu + m->nnu - 1] = 1.0;
    m->nsrc++;
    m->ltot = 0.0;
    for (int j = 0; j < m->nsrc; ++j) m->ltot += m->slum[j];
    double acc = 0.0;
    for (int j = 0; j < m->nsrc; ++j) {
        acc += m->slum[j];
        m->lcdf[j] = acc / m->ltot;
    }
    m->lcdf[m->nsrc - 1] = 1.0;
    return 0;
}

int orc_add_point_source(orc_model* m, const double pos[3], double lum, double teff)
{
    if (!m->have_nu) return fail(m, "set frequencies before sources");
    if (!(teff > 0.0)) return fail(m, "temperature must be > 0");
    double* lb = (double*)malloc(m->nnu * sizeof(double));
    for (int k = 0; k < m->nnu; ++k) lb[k] = orc_planck_bin(m->nu[k], m->nu[k + 1], teff);
    int r = add_source(m, pos, lum, lb);
    free(lb);
    return r;
}

int orc_add_point_source_spectrum(orc_model* m, const double pos[3], double lum,
                                  const double* l_nu_bin, int n_nu)
{
    if (!m->have_nu || n_nu != m->nnu) return fail(m, "spectrum size does not match the bins");
    return add_source(m, pos, lum, l_nu_bin);
}

int orc_set_observers(orc_model* m, int n_incl, int img_npix, double img_half_width,
                      const int* img_nu_bins, int n_img_nu)
{
    if (!m->have_nu) return fail(m, "set frequencies before observers");
    if (n_incl < 1) return fail(m, "need at least one inclination bin");
    if (n_img_nu < 0 || (n_img_nu > 0 && (img_npix < 1 || !(img_half_width > 0.0))))
        return fail(m, "bad image parameters");
    m->n_incl = n_incl;
    m->npix = n_img_nu > 0 ? img_npix : 0;
    m->n_img = n_img_nu;
    m->img_hw = img_half_width;
    free(m->img_bins); free(m->img_of_bin);
    m->img_bins = (int*)malloc((n_img_nu > 0 ? n_img_nu : 1) * sizeof(int));
    m->img_of_bin = (int*)malloc(m->nnu * sizeof(int));
    for (int k = 0; k < m->nnu; ++k) m->img_of_bin[k] = -1;
    for (int i = 0; i < n_img_nu; ++i) {
        if (img_nu_bins[i] < 0 || img_nu_bins[i] >= m->nnu) return fail(m, "image bin out of range");
        if (m->img_of_bin[img_nu_bins[i]] >= 0) return fail(m, "duplicate image bin");
        m->img_bins[i] = img_nu_bins[i];
        m->img_of_bin[img_nu_bins[i]] = i;
    }
    free(m->sed_sum); free(m->sed_sum2); free(m->sed_n); free(m->img_sum); free(m->img_sum2);
    size_t ns = (size_t)n_incl * m->nnu;
    size_t ni = (size_t)m->n_img * n_incl * m->npix * m->npix;
    m->sed_sum = (double*)calloc(ns, sizeof(double));
    m->sed_sum2 = (double*)calloc(ns, sizeof(double));
    m->sed_n = (int64_t*)calloc(ns, sizeof(int64_t));
    m->img_sum = (double*)calloc(ni ? ni : 1, sizeof(double));
    m->img_sum2 = (double*)calloc(ni ? ni : 1, sizeof(double));
    m->have_obs = 1;
    return 0;
}

int orc_set_peeloff(orc_model* m, const double* dirs, int n)
{
    if (!m->have_obs) return fail(m, "set observers before peeling-off directions");
    if (n < 0 || (n > 0 && !dirs)) return fail(m, "bad peeling-off directions");
    for (int i = 0; i < n; ++i) {
        double r = sqrt(dirs[3 * i] * dirs[3 * i] + dirs[3 * i + 1] * dirs[3 * i + 1] +
                        dirs[3 * i + 2] * dirs[3 * i + 2]);
        if (!(fabs(r - 1.0) < 1e-9)) return fail(m, "peeling-off directions must be unit vectors");
    }
    free(m->peel_dir); free(m->psed_sum); free(m->psed_sum2); free(m->pimg_sum); free(m->pimg_sum2);
    m->n_peel = n;
    size_t ns = (size_t)(n ? n : 1) * 2 * m->nnu;
    size_t ni = (size_t)m->n_img * (n ? n : 1) * m->npix * m->npix;
    m->peel_dir = (double*)malloc((size_t)(n ? n : 1) * 3 * sizeof(double));
    if (n) memcpy(m->peel_dir, dirs, (size_t)n * 3 * sizeof(double));
    m->psed_sum = (double*)calloc(ns, sizeof(double));
    m->psed_sum2 = (double*)calloc(ns, sizeof(double));
    m->pimg_sum = (double*)calloc(ni ? ni : 1, sizeof(double));
    m->pimg_sum2 = (double*)calloc(ni ? ni : 1, sizeof(double));
    return 0;
}

int orc_set_run(orc_model* m, const orc_run_cfg* cfg)
{
    if (cfg->n_packets < 1 || cfg->n_packets_final < 0) return fail(m, "packet counts must be >= 1");
    if (cfg->n_iter < 0) return fail(m, "n_iter must be >= 0");
    if (!(cfg->t_init > 0.0)) return fail(m, "t_init must be > 0");
    if (cfg->max_events < 0) return fail(m, "max_events must be >= 0");
    if (!(cfg->mrw_gamma >= 0.0)) return fail(m, "mrw_gamma must be >= 0");
    if (!(cfg->conv_p > 0.0 && cfg->conv_p <= 1.0)) return fail(m, "conv_p must be in (0,1]");
    if (cfg->event_log_packets < 0 || cfg->event_log_cap < 0) return fail(m, "bad event log size");
    m->cfg = *cfg;
    if (m->cfg.event_log_cap == 0) m->cfg.event_log_cap = 256;
    m->have_run = 1;
    return 0;
}

static int ensure_state(orc_model* m)
{
    if (m->T) return 0;
    size_t n = (size_t)m->ncell;
    m->T = (double*)malloc(n * sizeof(double));
    m->T_prev = (double*)malloc(n * sizeof(double));
    m->T_valid = (unsigned char*)malloc(n);
    m->sig_rel = (double*)calloc(n, sizeof(double));
    m->sig_rel_prev = (double*)calloc(n, sizeof(double));
    m->adot = (double*)calloc(n, sizeof(double));
    m->adot_prev = (double*)calloc(n, sizeof(double));
    m->adot_sig = (double*)calloc(n, sizeof(double));
    m->acc = (double*)calloc(n, sizeof(double));
    m->acc2 = (double*)calloc(n, sizeof(double));
    m->row_m = (int32_t*)malloc(n * sizeof(int32_t));
    m->row_w = (double*)malloc(n * sizeof(double));
    if (!m->T || !m->acc || !m->row_w) return fail(m, "out of memory");
    for (size_t j = 0; j < n; ++j) {
        m->T[j] = m->cfg.t_init;
        m->T_valid[j] = 1;
    }
    m->have_adot_prev = 0;
    m->q_prev = INFINITY;
    m->iter = 0;
    return 0;
}

int orc_set_temperature(orc_model* m, const double* T, size_t n)
{
    if (!m->have_grid || !m->have_run) return fail(m, "set grid and run parameters first");
    if ((int64_t)n != m->ncell) return fail(m, "temperature size does not match the grid");
    for (size_t j = 0; j < n; ++j)
        if (!(T[j] > 0.0) || !isfinite(T[j])) return fail(m, "temperature must be > 0");
    if (ensure_state(m)) return -1;
    memcpy(m->T, T, n * sizeof(double));
    for (size_t j = 0; j < n; ++j) {
        m->T_valid[j] = 1;
        m->sig_rel[j] = 0.0;
    }
    m->have_adot_prev = 0;
    m->q_prev = INFINITY;
    return 0;
}

/* ======================================================================= */
/* Sampling helpers.                                                       */
/* ======================================================================= */

/* smallest k with u < cdf[k]; cdf[n-1] == 1 */
static int cdf_search(const double* cdf, int n, double u)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi) / 2;
        if (u < cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

static void isotropic(double u_mu, double u_phi, double d[3])
{
    double mu = 2.0 * u_mu - 1.0;
    double phi = 2.0 * ORC_PI * u_phi;
    double s = sqrt(fmax(0.0, 1.0 - mu * mu));
    d[0] = s * cos(phi);
    d[1] = s * sin(phi);
    d[2] = mu;
}

void orc_isotropic(double u_mu, double u_phi, double d[3]) { isotropic(u_mu, u_phi, d); }

void orc_uniform_block(uint32_t key0, uint32_t key1, uint64_t packet0, int64_t n_packets,
                       int64_t n_draws, double* out)
{
    for (int64_t p = 0; p < n_packets; ++p)
        for (int64_t n = 0; n < n_draws; ++n)
            out[p * n_draws + n] = orc_uniform(key0, key1, packet0 + (uint64_t)p, (uint64_t)n);
}

/* Henyey-Greenstein: inverse of the cumulative distribution of mu = cos(theta) */
double orc_hg_mu(double g, double u)
{
    double mu;
    if (fabs(g) < 1e-6) {
        mu = 2.0 * u - 1.0;
    } else {
        double f = (1.0 - g * g) / (1.0 - g + 2.0 * g * u);
        mu = (1.0 + g * g - f * f) / (2.0 * g);
    }
    if (mu > 1.0) mu = 1.0;
    if (mu < -1.0) mu = -1.0;
    return mu;
}

/* New direction at angle acos(mu) from d and azimuth phi around d. */
void orc_rotate(const double d[3], double mu, double phi, double out[3])
{
    double st = sqrt(fmax(0.0, 1.0 - mu * mu));
    double cp = cos(phi), sp = sin(phi);
    if (fabs(d[2]) > 1.0 - 1e-10) {
        double sgn = d[2] > 0.0 ? 1.0 : -1.0;
        out[0] = st * cp;
        out[1] = st * sp;
        out[2] = sgn * mu;
    } else {
        double s = sqrt(1.0 - d[2] * d[2]);
        out[0] = st * (d[0] * d[2] * cp - d[1] * sp) / s + d[0] * mu;
        out[1] = st * (d[1] * d[2] * cp + d[0] * sp) / s + d[1] * mu;
        out[2] = -st * cp * s + d[2] * mu;
    }
    double nrm = sqrt(out[0] * out[0] + out[1] * out[1] + out[2] * out[2]);
    out[0] /= nrm;
    out[1] /= nrm;
    out[2] /= nrm;
}

static void locate(const orc_model* m, const double x[3], const double d[3], int c[3])
{
    for (int a = 0; a < 3; ++a) {
        double f = (x[a] - m->lo[a]) / m->dx[a];
        double fl = floor(f);
        int ci = (int)fl;
        if (f == fl && d[a] < 0.0) ci -= 1;
        c[a] = ci;
    }
}

static int inside(const orc_model* m, const int c[3])
{
    return c[0] >= 0 && c[0] < m->n[0] && c[1] >= 0 && c[1] < m->n[1] && c[2] >= 0 && c[2] < m->n[2];
}

static double wall(const orc_model* m, int a, int c) { return m->lo[a] + (double)c * m->dx[a]; }

/* distance along d to the wall that the packet in cell c reaches first on axis a */
static double wall_distance(const orc_model* m, const double x[3], const double d[3], const int c[3], int a)
{
    if (d[a] > 0.0) return (wall(m, a, c[a] + 1) - x[a]) / d[a];
    if (d[a] < 0.0) return (wall(m, a, c[a]) - x[a]) / d[a];
    return INFINITY;
}

/* ======================================================================= */
/* Per-thread tallies.                                                     */
/* ======================================================================= */
typedef struct {
    double* acc;
    double* acc2;
    double* sed_sum;
    double* sed_sum2;
    int64_t* sed_n;
    double* img_sum;
    double* img_sum2;
    double* psed_sum;
    double* psed_sum2;
    double* pimg_sum;
    double* pimg_sum2;
    int64_t n_cross_dust, n_cross_empty, n_scatter, n_absorb, n_escape, n_killed, n_mrw;
    double e_escaped, e_killed;
} tally;

static void log_event(const orc_model* m, int64_t p, int type, const int c[3], int k, int incl)
{
    int64_t q = p - m->ev_first; /* slot of the packet in the log */
    if (q < 0 || q >= m->ev_packets) return;
    int32_t i = m->evcount[q];
    if (i < m->ev_cap) {
        orc_event* e = m->evlog + (size_t)q * m->ev_cap + i;
        e->packet = p;
        e->index = i;
        e->type = type;
        e->cell[0] = c[0]; e->cell[1] = c[1]; e->cell[2] = c[2];
        e->nu = k;
        e->incl = incl;
        e->reserved = 0;
    }
    m->evcount[q] = i + 1;
}

/*
 * Walk the grid from x in cell c along d with frequency bin k until the
 * optical depth tau is used up (returns 1, x at the interaction point, c its
 * cell) or the packet leaves the grid (returns 0, x on the boundary, c the
 * last cell inside).  Every segment in a dust cell adds eps*l*kappa_k to that
 * cell's absorption tally (Eq. 2).
 */
static int walk(const orc_model* m, double x[3], const double d[3], int c[3], int k, double tau,
                double eps, tally* t)
{
    double tau_acc = 0.0;
    const double chi = m->chi[k], kap = m->kap[k];
    for (;;) {
        int64_t j = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
        double tw[3];
        for (int a = 0; a < 3; ++a) tw[a] = wall_distance(m, x, d, c, a);
        int ax = 0;
        if (tw[1] < tw[ax]) ax = 1;
        if (tw[2] < tw[ax]) ax = 2;
        double l = tw[ax] > 0.0 ? tw[ax] : 0.0;
        double rho = m->rho[j];
        if (rho > 0.0) {
            t->n_cross_dust++;
            double dtau = rho * chi * l;
            if (tau_acc + dtau >= tau) {
                double lp = (tau - tau_acc) / (rho * chi);
                double w = eps * lp * kap;
                t->acc[j] += w;
                if (t->acc2) t->acc2[j] += w * w;
                for (int a = 0; a < 3; ++a) x[a] += d[a] * lp;
                return 1;
            }
            double w = eps * l * kap;
            t->acc[j] += w;
            if (t->acc2) t->acc2[j] += w * w;
            tau_acc += dtau;
        } else {
            t->n_cross_empty++;
        }
        for (int a = 0; a < 3; ++a) x[a] += d[a] * l;
        if (d[ax] > 0.0) {
            x[ax] = wall(m, ax, c[ax] + 1);
            if (c[ax] + 1 >= m->n[ax]) return 0;
            c[ax] += 1;
        } else {
            x[ax] = wall(m, ax, c[ax]);
            if (c[ax] - 1 < 0) return 0;
            c[ax] -= 1;
        }
    }
}

static void bin_escape(const orc_model* m, const double x[3], const double d[3], int k, double eps,
                       int incl, tally* t)
{
    size_t s = (size_t)incl * m->nnu + k;
    t->sed_sum[s] += eps;
    t->sed_sum2[s] += eps * eps;
    t->sed_n[s] += 1;
    int ii = m->img_of_bin[k];
    if (ii < 0) return;
    double p[3];
    for (int a = 0; a < 3; ++a) p[a] = x[a] - 0.5 * (m->lo[a] + m->hi[a]);
    double ex[3] = {-d[1], d[0], 0.0};
    double en = sqrt(ex[0] * ex[0] + ex[1] * ex[1]);
    if (en < 1e-12) {
        ex[0] = 1.0; ex[1] = 0.0;
    } else {
        ex[0] /= en; ex[1] /= en;
    }
    double ey[3] = {d[1] * ex[2] - d[2] * ex[1], d[2] * ex[0] - d[0] * ex[2], d[0] * ex[1] - d[1] * ex[0]};
    double X = p[0] * ex[0] + p[1] * ex[1] + p[2] * ex[2];
    double Y = p[0] * ey[0] + p[1] * ey[1] + p[2] * ey[2];
    double fx = floor((X + m->img_hw) / (2.0 * m->img_hw) * m->npix);
    double fy = floor((Y + m->img_hw) / (2.0 * m->img_hw) * m->npix);
    if (fx < 0.0 || fy < 0.0 || fx >= m->npix || fy >= m->npix) return;
    size_t q = (((size_t)ii * m->n_incl + incl) * m->npix + (size_t)fy) * m->npix + (size_t)fx;
    t->img_sum[q] += eps;
    t->img_sum2[q] += eps * eps;
}

/* Optical depth in bin k from x to the grid boundary along the unit vector
 * o: the same walk as for a packet, without interactions.  0 when x lies
 * outside the grid. */
static double tau_to_boundary(const orc_model* m, const double x0[3], const double o[3], int k)
{
    double x[3] = {x0[0], x0[1], x0[2]};
    int c[3];
    locate(m, x, o, c);
    if (!inside(m, c)) return 0.0;
    double tau = 0.0;
    for (;;) {
        int64_t j = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
        double tw[3];
        for (int a = 0; a < 3; ++a) tw[a] = wall_distance(m, x, o, c, a);
        int ax = 0;
        if (tw[1] < tw[ax]) ax = 1;
        if (tw[2] < tw[ax]) ax = 2;
        double l = tw[ax] > 0.0 ? tw[ax] : 0.0;
        tau += m->rho[j] * m->chi[k] * l;
        for (int a = 0; a < 3; ++a) x[a] += o[a] * l;
        if (o[ax] > 0.0) {
            x[ax] = wall(m, ax, c[ax] + 1);
            if (c[ax] + 1 >= m->n[ax]) return tau;
            c[ax] += 1;
        } else {
            x[ax] = wall(m, ax, c[ax]);
            if (c[ax] - 1 < 0) return tau;
            c[ax] -= 1;
        }
    }
}

/* Henyey-Greenstein phase function per steradian (integrates to 1). */
static double hg_phase(double g, double mu)
{
    double q = 1.0 + g * g - 2.0 * g * mu;
    return (1.0 - g * g) / (4.0 * ORC_PI * q * sqrt(q));
}

/* Peeling-off (Sec. 2.6.2): toward every observer o, add eps * p(o) *
 * exp(-tau(x -> boundary along o)) in bin k to the SED component comp and,
 * for the image bins, to the pixel of x projected along o.  d_in is the
 * incoming direction of a scattering (p from the HG phase function) or NULL
 * for isotropic emission (p = 1/(4 pi)). */
static void peel(const orc_model* m, const double x[3], const double* d_in, int k, double eps, int comp,
                 tally* t)
{
    for (int i = 0; i < m->n_peel; ++i) {
        const double* o = m->peel_dir + 3 * i;
        double p = 1.0 / (4.0 * ORC_PI);
        if (d_in) p = hg_phase(m->g[k], d_in[0] * o[0] + d_in[1] * o[1] + d_in[2] * o[2]);
        double w = eps * p * exp(-tau_to_boundary(m, x, o, k));
        size_t q = ((size_t)i * 2 + comp) * m->nnu + k;
        t->psed_sum[q] += w;
        t->psed_sum2[q] += w * w;
        int ii = m->img_of_bin[k];
        if (ii < 0) continue;
        double pc[3];
        for (int a = 0; a < 3; ++a) pc[a] = x[a] - 0.5 * (m->lo[a] + m->hi[a]);
        double ex[3] = {-o[1], o[0], 0.0};
        double en = sqrt(ex[0] * ex[0] + ex[1] * ex[1]);
        if (en < 1e-12) {
            ex[0] = 1.0; ex[1] = 0.0;
        } else {
            ex[0] /= en; ex[1] /= en;
        }
        double ey[3] = {o[1] * ex[2] - o[2] * ex[1], o[2] * ex[0] - o[0] * ex[2], o[0] * ex[1] - o[1] * ex[0]};
        double X = pc[0] * ex[0] + pc[1] * ex[1] + pc[2] * ex[2];
        double Y = pc[0] * ey[0] + pc[1] * ey[1] + pc[2] * ey[2];
        double fx = floor((X + m->img_hw) / (2.0 * m->img_hw) * m->npix);
        double fy = floor((Y + m->img_hw) / (2.0 * m->img_hw) * m->npix);
        if (fx < 0.0 || fy < 0.0 || fx >= m->npix || fy >= m->npix) continue;
        size_t r = (((size_t)ii * m->n_peel + i) * m->npix + (size_t)fy) * m->npix + (size_t)fx;
        t->pimg_sum[r] += w;
        t->pimg_sum2[r] += w * w;
    }
}

/* ======================================================================= */
/* Modified random walk (Sec. 2.2).                                         */
/* ======================================================================= */
/* The paper names the method (Min et al. 2009, in the form of Robitaille 2010)
 * without its steps; they are taken here from diffusion in a sphere.  A
 * packet at x in a cell of density rho whose nearest wall is R0 away, with
 * rho chi_R R0 >= gamma (chi_R the Rosseland mean at the cell's T), diffuses
 * with coefficient D = 1/(3 rho chi_R) (per unit path length) from the centre
 * of the sphere of radius R0; the path length s until it first reaches the
 * sphere has the distribution of first-passage times of diffusion from the
 * centre, F(y) = 1 + 2 sum_{n>=1} (-1)^n exp(-n^2 y), y = pi^2 D s / R0^2.
 * The step moves x to a uniformly random point of the sphere, adds
 * eps kappa_P s to the cell's path-length tally (the estimator of Eq. 2 with
 * the Planck-mean absorption of the cell's T: the radiation inside an
 * optically thick cell is thermal), and re-emits the packet in a bin drawn
 * from the cell's emissivity, in an isotropic direction.  Steps repeat while
 * the condition holds; each counts as an interaction. */
double orc_mrw_escape_cdf(double y)
{
    if (!(y > 0.0)) return 0.0;
    double f = 0.0;
    if (y < 2.0) {
        /* the same function after Jacobi's transformation (fast for small y) */
        for (int m = 0; m < 50; ++m) {
            double a = (2.0 * m + 1.0) * ORC_PI;
            double term = exp(-a * a / (4.0 * y));
            f += term;
            if (term < 1e-300) break;
        }
        return 2.0 * sqrt(ORC_PI / y) * f;
    }
    double sgn = -1.0;
    for (int n = 1; n < 50; ++n) {
        double term = exp(-(double)n * n * y);
        f += sgn * term;
        sgn = -sgn;
        if (term < 1e-300) break;
    }
    return 1.0 + 2.0 * f;
}

double orc_mrw_escape_y(double u)
{
    double lo = 1e-3, hi = 80.0; /* F(1e-3) ~ 1e-1070, 1 - F(80) ~ 1e-34 */
    for (int i = 0; i < 200; ++i) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (orc_mrw_escape_cdf(mid) < u) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

double orc_planck_mean_kappa(const orc_model* m, double T)
{
    double num = 0.0, den = 0.0;
    for (int k = 0; k < m->nnu; ++k) {
        double b = orc_planck_bin(m->nu[k], m->nu[k + 1], T);
        num += m->kap[k] * b;
        den += b;
    }
    return den > 0.0 ? num / den : 0.0;
}

/* int_a^b x^4 e^x / (e^x - 1)^2 dx by composite Simpson (step <= 0.01); the
 * integrand beyond x = 60 holds less than 1e-20 of the total and is left out */
static double dplanck_x_integral(double a, double b)
{
    if (a > 60.0) return 0.0;
    if (b > 60.0) b = 60.0;
    int n = (int)ceil((b - a) / 0.01);
    if (n < 8) n = 8;
    if (n % 2) n += 1;
    double h = (b - a) / n, s = 0.0;
    for (int i = 0; i <= n; ++i) {
        double x = a + i * h;
        double sh = sinh(0.5 * x);
        double f = x > 0.0 ? x * x * x * x / (4.0 * sh * sh) : 0.0;
        s += f * (i == 0 || i == n ? 1.0 : (i % 2 ? 4.0 : 2.0));
    }
    return s * h / 3.0;
}

double orc_rosseland_chi(const orc_model* m, double T)
{
    /* 1/chi_R = sum_k (1/chi_k) dB_k/dT / sum_k dB_k/dT; the common factor
     * 2 k^4 T^3 / (h^3 c^2) of dB_k/dT cancels */
    double kT = ORC_K_BOLTZ * T, num = 0.0, den = 0.0;
    for (int k = 0; k < m->nnu; ++k) {
        double w = dplanck_x_integral(ORC_H_PLANCK * m->nu[k] / kT, ORC_H_PLANCK * m->nu[k + 1] / kT);
        num += w / m->chi[k];
        den += w;
    }
    return num > 0.0 ? den / num : INFINITY;
}

/* Modified-random-walk steps from x in cell c (see above); returns 1 when
 * the packet was killed at the event limit. */
static int mrw(const orc_model* m, orc_stream* rs, int64_t p, double x[3], double d[3], const int c[3],
               int* k, double eps, int peeling, int64_t* nev, tally* t)
{
    const int64_t j = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
    const double r = m->rho[j];
    if (!(r > 0.0)) return 0;
    const double chir = m->mrw_chir[j], kp = m->mrw_kp[j];
    for (;;) {
        double R0 = INFINITY;
        for (int a = 0; a < 3; ++a) {
            double dl = x[a] - wall(m, a, c[a]), dh = wall(m, a, c[a] + 1) - x[a];
            if (dl < R0) R0 = dl;
            if (dh < R0) R0 = dh;
        }
        if (!(r * chir * R0 >= m->cfg.mrw_gamma)) return 0;
        (*nev)++;
        if (*nev > m->cfg.max_events) {
            t->n_killed++;
            t->e_killed += eps;
            log_event(m, p, EV_KILLED, c, *k, -1);
            return 1;
        }
        double u_y = draw(rs), u_mu = draw(rs), u_phi = draw(rs), u_mix = draw(rs), u_nu = draw(rs);
        double u_mu2 = draw(rs), u_phi2 = draw(rs);
        double y = orc_mrw_escape_y(u_y);
        double s = 3.0 * r * chir * R0 * R0 * y / (ORC_PI * ORC_PI);
        double w = eps * kp * s;
        t->acc[j] += w;
        if (t->acc2) t->acc2[j] += w * w;
        double u[3];
        isotropic(u_mu, u_phi, u);
        for (int a = 0; a < 3; ++a) x[a] += R0 * u[a];
#ifdef ORC_MRW_NUDGE
        /* sensitivity experiment only (a separate test build): move the point
         * by one unit in the last place after every step */
        for (int a = 0; a < 3; ++a) x[a] = nextafter(x[a], INFINITY);
#endif
        int row = m->row_m[j] + (u_mix < m->row_w[j] ? 1 : 0);
        *k = cdf_search(m->ecdf + (size_t)row * m->nnu, m->nnu, u_nu);
        isotropic(u_mu2, u_phi2, d);
        t->n_mrw++;
        log_event(m, p, EV_MRW, c, *k, -1);
        if (peeling) peel(m, x, NULL, *k, eps, 1, t);
    }
}

/* Follow one source packet from emission to escape or kill (Sec. 2.2). */
static void run_packet(const orc_model* m, uint32_t key1, int64_t p, int64_t np, int binning, tally* t)
{
    orc_stream rs = {(uint32_t)(m->cfg.seed & 0xffffffffu), key1, (uint64_t)p, 0};
    double u_src = draw(&rs), u_nu = draw(&rs), u_mu = draw(&rs), u_phi = draw(&rs);
    int s;
    double eps;
    if (m->cfg.source_sampling == 0) {
        s = cdf_search(m->lcdf, m->nsrc, u_src);
        eps = m->ltot / (double)np;
    } else {
        s = (int)(p % m->nsrc);
        int64_t ns = np / m->nsrc + ((p % m->nsrc) < (np % m->nsrc) ? 1 : 0);
        eps = m->slum[s] / (double)ns;
    }
    int k = cdf_search(m->scdf + (size_t)s * m->nnu, m->nnu, u_nu);
    double d[3], x[3];
    isotropic(u_mu, u_phi, d);
    for (int a = 0; a < 3; ++a) x[a] = m->spos[3 * s + a];
    int c[3];
    locate(m, x, d, c);
    log_event(m, p, EV_EMIT, c, k, -1);
    const int peeling = binning && m->n_peel > 0;
    if (peeling) peel(m, x, NULL, k, eps, 0, t);
    int64_t nev = 0;
    int in = inside(m, c);
    for (;;) {
        if (in && m->cfg.mrw_gamma > 0.0 && mrw(m, &rs, p, x, d, c, &k, eps, peeling, &nev, t)) return;
        double tau = -log(draw(&rs));
        int hit = in ? walk(m, x, d, c, k, tau, eps, t) : 0;
        if (!hit) {
            int incl = (int)(fabs(d[2]) * m->n_incl);
            if (incl >= m->n_incl) incl = m->n_incl - 1;
            t->n_escape++;
            t->e_escaped += eps;
            if (binning) bin_escape(m, x, d, k, eps, incl, t);
            log_event(m, p, EV_ESCAPE, c, k, incl);
            return;
        }
        nev++;
        if (nev > m->cfg.max_events) {
            t->n_killed++;
            t->e_killed += eps;
            log_event(m, p, EV_KILLED, c, k, -1);
            return;
        }
        double u_int = draw(&rs);
        int64_t j = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
        if (u_int > m->alb[k]) {
            double u_mix = draw(&rs), u_nu2 = draw(&rs), u_mu2 = draw(&rs), u_phi2 = draw(&rs);
            int row = m->row_m[j] + (u_mix < m->row_w[j] ? 1 : 0);
            k = cdf_search(m->ecdf + (size_t)row * m->nnu, m->nnu, u_nu2);
            isotropic(u_mu2, u_phi2, d);
            t->n_absorb++;
            log_event(m, p, EV_ABSORB, c, k, -1);
            if (peeling) peel(m, x, NULL, k, eps, 1, t);
        } else {
            double u_mu2 = draw(&rs), u_phi2 = draw(&rs);
            double mu = orc_hg_mu(m->g[k], u_mu2);
            double dn[3];
            if (peeling) peel(m, x, d, k, eps, 1, t);
            orc_rotate(d, mu, 2.0 * ORC_PI * u_phi2, dn);
            d[0] = dn[0]; d[1] = dn[1]; d[2] = dn[2];
            t->n_scatter++;
            log_event(m, p, EV_SCATTER, c, k, -1);
        }
    }
}

static double now_seconds(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int ready(orc_model* m)
{
    if (!m->have_grid || !m->have_rho) return fail(m, "grid and density must be set");
    if (!m->have_dust) return fail(m, "dust must be set");
    if (m->nsrc < 1) return fail(m, "add at least one source");
    if (!m->have_run) return fail(m, "run parameters must be set");
    if (!m->have_obs) {
        if (orc_set_observers(m, 10, 0, 0.0, NULL, 0)) return -1;
    }
    return ensure_state(m);
}

/* Emission row and weight of every cell from its temperature (reading of Sec. 2.1.3). */
static int64_t rows_from_T(orc_model* m)
{
    int64_t clamped = 0;
    const double lr = log(ORC_T_HI / ORC_T_LO);
    for (int64_t j = 0; j < m->ncell; ++j) {
        double T = m->T[j];
        double p = (double)(ORC_NROW - 1) * log(T / ORC_T_LO) / lr;
        if (T < ORC_T_LO || T > ORC_T_HI) clamped += m->rho[j] > 0.0;
        if (p < 0.0) p = 0.0;
        if (p > (double)(ORC_NROW - 1)) p = (double)(ORC_NROW - 1);
        int r = (int)floor(p);
        if (r > ORC_NROW - 2) r = ORC_NROW - 2;
        double w = p - (double)r;
        m->row_m[j] = r;
        m->row_w[j] = w;
    }
    if (m->cfg.mrw_gamma > 0.0) {
        if (!m->mrw_kp) {
            m->mrw_kp = (double*)calloc((size_t)m->ncell, sizeof(double));
            m->mrw_chir = (double*)calloc((size_t)m->ncell, sizeof(double));
        }
        for (int64_t j = 0; j < m->ncell; ++j) {
            if (!(m->rho[j] > 0.0)) continue;
            m->mrw_kp[j] = orc_planck_mean_kappa(m, m->T[j]);
            m->mrw_chir[j] = orc_rosseland_chi(m, m->T[j]);
        }
    }
    return clamped;
}

/*
 * Propagate np packets with Philox key word key1, in chunks spread over the
 * threads; each thread owns private tallies that are summed in thread order
 * afterwards (results are independent of the partition up to the order of
 * floating-point summation, Sec. 3).
 */
static int transport(orc_model* m, int64_t np, int64_t p_first, int64_t p_count, uint32_t key1,
                     int binning, orc_iter_stats* st)
{
    int nt = 1;
#ifdef _OPENMP
    nt = m->cfg.n_threads > 0 ? m->cfg.n_threads : omp_get_max_threads();
#endif
    int64_t chunk = m->cfg.chunk > 0 ? m->cfg.chunk : 1024;
    int64_t nchunk = (p_count + chunk - 1) / chunk;
    size_t nc = (size_t)m->ncell;
    size_t ns = (size_t)m->n_incl * m->nnu;
    size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    size_t nps = (size_t)m->n_peel * 2 * m->nnu;
    size_t npi = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    tally* T = (tally*)calloc(nt, sizeof(tally));
    for (int i = 0; i < nt; ++i) {
        T[i].acc = (double*)calloc(nc, sizeof(double));
        T[i].acc2 = m->cfg.want_noise ? (double*)calloc(nc, sizeof(double)) : NULL;
        T[i].sed_sum = (double*)calloc(ns, sizeof(double));
        T[i].sed_sum2 = (double*)calloc(ns, sizeof(double));
        T[i].sed_n = (int64_t*)calloc(ns, sizeof(int64_t));
        T[i].img_sum = (double*)calloc(ni ? ni : 1, sizeof(double));
        T[i].img_sum2 = (double*)calloc(ni ? ni : 1, sizeof(double));
        T[i].psed_sum = (double*)calloc(nps ? nps : 1, sizeof(double));
        T[i].psed_sum2 = (double*)calloc(nps ? nps : 1, sizeof(double));
        T[i].pimg_sum = (double*)calloc(npi ? npi : 1, sizeof(double));
        T[i].pimg_sum2 = (double*)calloc(npi ? npi : 1, sizeof(double));
        if (!T[i].acc || !T[i].img_sum2 || !T[i].pimg_sum2) return fail(m, "out of memory");
    }
    /* event log */
    free(m->evlog); free(m->evcount);
    m->ev_packets = (int)(m->cfg.event_log_packets < p_count ? m->cfg.event_log_packets : p_count);
    m->ev_first = p_first;
    m->ev_cap = m->cfg.event_log_cap;
    m->evlog = (orc_event*)calloc((size_t)(m->ev_packets ? m->ev_packets : 1) * m->ev_cap, sizeof(orc_event));
    m->evcount = (int32_t*)calloc(m->ev_packets ? m->ev_packets : 1, sizeof(int32_t));

    double t0 = now_seconds();
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t ch = 0; ch < nchunk; ++ch) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        int64_t p1 = (ch + 1) * chunk < p_count ? (ch + 1) * chunk : p_count;
        for (int64_t p = ch * chunk; p < p1; ++p)
            run_packet(m, key1, p_first + p, np, binning, &T[tid]);
    }
    double t1 = now_seconds();

    /* reduce in thread order */
    for (size_t j = 0; j < nc; ++j) {
        double a = 0.0, a2 = 0.0;
        for (int i = 0; i < nt; ++i) {
            a += T[i].acc[j];
            if (T[i].acc2) a2 += T[i].acc2[j];
        }
        m->acc[j] += a;
        m->acc2[j] += a2;
    }
    for (int i = 0; i < nt; ++i) {
        for (size_t s = 0; s < ns; ++s) {
            m->sed_sum[s] += T[i].sed_sum[s];
            m->sed_sum2[s] += T[i].sed_sum2[s];
            m->sed_n[s] += T[i].sed_n[s];
        }
        for (size_t q = 0; q < ni; ++q) {
            m->img_sum[q] += T[i].img_sum[q];
            m->img_sum2[q] += T[i].img_sum2[q];
        }
        for (size_t q = 0; q < nps; ++q) {
            m->psed_sum[q] += T[i].psed_sum[q];
            m->psed_sum2[q] += T[i].psed_sum2[q];
        }
        for (size_t q = 0; q < npi; ++q) {
            m->pimg_sum[q] += T[i].pimg_sum[q];
            m->pimg_sum2[q] += T[i].pimg_sum2[q];
        }
        st->n_cross_dust += T[i].n_cross_dust;
        st->n_cross_empty += T[i].n_cross_empty;
        st->n_scatter += T[i].n_scatter;
        st->n_absorb += T[i].n_absorb;
        st->n_escape += T[i].n_escape;
        st->n_killed += T[i].n_killed;
        st->n_mrw += T[i].n_mrw;
        st->e_escaped += T[i].e_escaped;
        st->e_killed += T[i].e_killed;
        free(T[i].acc); free(T[i].acc2); free(T[i].sed_sum); free(T[i].sed_sum2); free(T[i].sed_n);
        free(T[i].img_sum); free(T[i].img_sum2);
        free(T[i].psed_sum); free(T[i].psed_sum2); free(T[i].pimg_sum); free(T[i].pimg_sum2);
    }
    free(T);
    st->seconds = t1 - t0;
    return 0;
}

/* ======================================================================= */
/* Temperature (Eq. 3 over the model's bins).                              */
/* ======================================================================= */

/* F(T) = 4 pi sum_k kappa_k B_k(T), and dlnF/dlnT */
static double adot_and_slope(const orc_model* m, double T, double* slope)
{
    double kT = ORC_K_BOLTZ * T;
    double pref = 2.0 * pow(kT, 4) / (pow(ORC_H_PLANCK, 3) * ORC_C_LIGHT * ORC_C_LIGHT);
    double s = 0.0, ds = 0.0;
    for (int k = 0; k < m->nnu; ++k) {
        if (m->kap[k] == 0.0) continue;
        double a = ORC_H_PLANCK * m->nu[k] / kT;
        double b = ORC_H_PLANCK * m->nu[k + 1] / kT;
        double I = orc_planck_x_integral(a, b);
        s += m->kap[k] * I;
        /* d/dT [T^4 I(a(T), b(T))] = T^3 (4 I + a f(a) - b f(b)) */
        ds += m->kap[k] * (4.0 * I + a * planck_f(a) - b * planck_f(b));
    }
    if (slope) *slope = s > 0.0 ? ds / s : 4.0;
    return 4.0 * ORC_PI * pref * s;
}

double orc_adot_of_T(const orc_model* m, double T) { return adot_and_slope(m, T, NULL); }

/* Safeguarded Newton iteration in y = ln T on the bracket [ln 1 K, ln 1e4 K]. */
double orc_solve_T(const orc_model* m, double adot, int* clamped)
{
    if (clamped) *clamped = 0;
    double flo = adot_and_slope(m, ORC_T_LO, NULL);
    double fhi = adot_and_slope(m, ORC_T_HI, NULL);
    if (adot <= flo) {
        if (clamped) *clamped = adot < flo;
        return ORC_T_LO;
    }
    if (adot >= fhi) {
        if (clamped) *clamped = adot > fhi;
        return ORC_T_HI;
    }
    double ya = log(ORC_T_LO), yb = log(ORC_T_HI);
    double target = log(adot);
    double y = ya + (yb - ya) * (target - log(flo)) / (log(fhi) - log(flo));
    for (int it = 0; it < 200; ++it) {
        double slope;
        double F = adot_and_slope(m, exp(y), &slope);
        double gres = log(F) - target;
        if (gres > 0.0) yb = y;
        else ya = y;
        double yn = y - gres / slope;
        if (!(yn > ya && yn < yb)) yn = 0.5 * (ya + yb);
        if (fabs(yn - y) <= 1e-15 * fabs(y) + 1e-300 || yb - ya < 1e-15) {
            y = yn;
            break;
        }
        y = yn;
    }
    return exp(y);
}

static int cmp_double(const void* a, const void* b)
{
    double x = *(const double*)a, y = *(const double*)b;
    return (x > y) - (x < y);
}

double orc_percentile(const double* v, int64_t n, double p)
{
    if (n <= 0) return NAN;
    double* s = (double*)malloc((size_t)n * sizeof(double));
    memcpy(s, v, (size_t)n * sizeof(double));
    qsort(s, (size_t)n, sizeof(double), cmp_double);
    int64_t r = (int64_t)ceil(p * (double)n);
    if (r < 1) r = 1;
    if (r > n) r = n;
    double q = s[r - 1];
    free(s);
    return q;
}

static double delta_ratio(double a, double b) { return a > b ? a / b : b / a; } /* Eq. 4 */

/* Ȧ, T and the convergence statistics after the transport of an iteration. */
static void finish_iteration(orc_model* m, orc_iter_stats* st)
{
    int64_t nc = m->ncell;
    memcpy(m->T_prev, m->T, (size_t)nc * sizeof(double));
    memcpy(m->sig_rel_prev, m->sig_rel, (size_t)nc * sizeof(double));
    unsigned char* valid_prev = (unsigned char*)malloc((size_t)nc);
    memcpy(valid_prev, m->T_valid, (size_t)nc);
    int64_t n_uns = 0, n_cl = 0;
#ifdef _OPENMP
    int nt = m->cfg.n_threads > 0 ? m->cfg.n_threads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : n_uns, n_cl) num_threads(nt)
#endif
    for (int64_t j = 0; j < nc; ++j) {
        double a = m->acc[j] / m->vol; /* Eq. 2 with Delta t = 1 s */
        m->adot[j] = a;
        m->adot_sig[j] = sqrt(m->acc2[j]) / m->vol;
        if (a > 0.0) {
            int cl = 0;
            double T = orc_solve_T(m, a, &cl);
            n_cl += cl;
            double slope = 4.0;
            if (m->cfg.want_noise) adot_and_slope(m, T, &slope);
            m->T[j] = T;
            m->T_valid[j] = 1;
            /* sigma_T/T = (sigma_Ȧ/Ȧ) dlnT/dlnȦ */
            m->sig_rel[j] = m->cfg.want_noise ? (m->adot_sig[j] / a) / slope : 0.0;
        } else {
            m->T[j] = ORC_T_FLOOR;
            m->T_valid[j] = 0;
            m->sig_rel[j] = 0.0;
            if (m->rho[j] > 0.0) n_uns++;
        }
    }
    st->n_unsampled = n_uns;
    st->n_t_clamped = n_cl;

    /* Eqs. 4-6 on Ȧ */
    double* R = (double*)malloc((size_t)nc * sizeof(double));
    int64_t nr = 0;
    if (m->have_adot_prev) {
        for (int64_t j = 0; j < nc; ++j)
            if (m->rho[j] > 0.0 && m->adot_prev[j] > 0.0 && m->adot[j] > 0.0)
                R[nr++] = delta_ratio(m->adot_prev[j], m->adot[j]);
    }
    st->n_r = nr;
    st->q = nr > 0 ? orc_percentile(R, nr, m->cfg.conv_p) : INFINITY;
    st->delta = (isfinite(st->q) && isfinite(m->q_prev)) ? delta_ratio(m->q_prev, st->q) : INFINITY;
    st->converged_q = st->q < m->cfg.conv_q_thres && st->delta < m->cfg.conv_d_thres;
    m->q_prev = st->q;

    /* max |dT/T| over the mask (reading of the max dT/T < 1 % criterion) */
    int64_t nm = 0;
    for (int64_t j = 0; j < nc; ++j) {
        if (!(m->rho[j] > 0.0 && m->adot[j] > 0.0 && valid_prev[j])) continue;
        if (m->cfg.want_noise) {
            double s2 = m->sig_rel[j] * m->sig_rel[j] + m->sig_rel_prev[j] * m->sig_rel_prev[j];
            if (sqrt(s2) > 0.002) continue;
        }
        R[nm++] = fabs(m->T[j] - m->T_prev[j]) / m->T_prev[j];
    }
    st->n_mask = nm;
    double mx = 0.0;
    for (int64_t i = 0; i < nm; ++i) mx = R[i] > mx ? R[i] : mx;
    st->max_dT = nm > 0 ? mx : INFINITY;
    st->p999_dT = nm > 0 ? orc_percentile(R, nm, 0.999) : INFINITY;
    st->converged_dT = nm > 0 && mx < m->cfg.conv_dT_thres;
    free(R);
    free(valid_prev);
    memcpy(m->adot_prev, m->adot, (size_t)nc * sizeof(double));
    m->have_adot_prev = 1;
}

static void clear_bins(orc_model* m)
{
    size_t ns = (size_t)m->n_incl * m->nnu;
    size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    memset(m->sed_sum, 0, ns * sizeof(double));
    memset(m->sed_sum2, 0, ns * sizeof(double));
    memset(m->sed_n, 0, ns * sizeof(int64_t));
    if (ni) {
        memset(m->img_sum, 0, ni * sizeof(double));
        memset(m->img_sum2, 0, ni * sizeof(double));
    }
    size_t nps = (size_t)m->n_peel * 2 * m->nnu;
    size_t npi = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    if (nps) {
        memset(m->psed_sum, 0, nps * sizeof(double));
        memset(m->psed_sum2, 0, nps * sizeof(double));
    }
    if (npi) {
        memset(m->pimg_sum, 0, npi * sizeof(double));
        memset(m->pimg_sum2, 0, npi * sizeof(double));
    }
}

int orc_iterate(orc_model* m, orc_iter_stats* st)
{
    if (ready(m)) return -1;
    memset(st, 0, sizeof *st);
    st->n_row_clamped = rows_from_T(m);
    memset(m->acc, 0, (size_t)m->ncell * sizeof(double));
    memset(m->acc2, 0, (size_t)m->ncell * sizeof(double));
    if (m->cfg.bin_every_iteration) clear_bins(m);
    if (transport(m, m->cfg.n_packets, 0, m->cfg.n_packets, (uint32_t)m->iter,
                  m->cfg.bin_every_iteration, st))
        return -1;
    finish_iteration(m, st);
    st->iteration = m->iter;
    m->iter++;
    return 0;
}

int orc_final_pass(orc_model* m, orc_iter_stats* st)
{
    if (ready(m)) return -1;
    memset(st, 0, sizeof *st);
    st->n_row_clamped = rows_from_T(m);
    memset(m->acc, 0, (size_t)m->ncell * sizeof(double));
    memset(m->acc2, 0, (size_t)m->ncell * sizeof(double));
    clear_bins(m);
    int64_t np = m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets;
    if (transport(m, np, 0, np, 0x80000000u | (uint32_t)m->iter, 1, st)) return -1;
    st->iteration = m->iter;
    return 0;
}

int orc_transport_sample(orc_model* m, int64_t n_packets, orc_iter_stats* st)
{
    if (ready(m)) return -1;
    if (n_packets < 1) return fail(m, "n_packets must be >= 1");
    memset(st, 0, sizeof *st);
    st->n_row_clamped = rows_from_T(m);
    memset(m->acc, 0, (size_t)m->ncell * sizeof(double));
    memset(m->acc2, 0, (size_t)m->ncell * sizeof(double));
    if (transport(m, n_packets, 0, n_packets, (uint32_t)m->iter, 0, st)) return -1;
    st->iteration = m->iter;
    return 0;
}

int orc_transport_range(orc_model* m, int64_t np_total, int64_t p_first, int64_t p_count,
                        int final_pass, orc_iter_stats* st)
{
    if (ready(m)) return -1;
    if (np_total < 1 || p_first < 0 || p_count < 0 || p_first + p_count > np_total)
        return fail(m, "bad packet range");
    memset(st, 0, sizeof *st);
    st->n_row_clamped = rows_from_T(m);
    memset(m->acc, 0, (size_t)m->ncell * sizeof(double));
    memset(m->acc2, 0, (size_t)m->ncell * sizeof(double));
    clear_bins(m);
    uint32_t key1 = final_pass ? (0x80000000u | (uint32_t)m->iter) : (uint32_t)m->iter;
    if (transport(m, np_total, p_first, p_count, key1, final_pass, st)) return -1;
    st->iteration = m->iter;
    return 0;
}

/* ======================================================================= */
/* Results.                                                                */
/* ======================================================================= */
int orc_get_specific_energy(const orc_model* m, double* adot, double* adot_sigma, size_t n)
{
    if (!m->adot || (int64_t)n != m->ncell) return -1;
    memcpy(adot, m->adot, n * sizeof(double));
    if (adot_sigma) memcpy(adot_sigma, m->adot_sig, n * sizeof(double));
    return 0;
}

int orc_get_temperature(const orc_model* m, double* T, size_t n)
{
    if (!m->T || (int64_t)n != m->ncell) return -1;
    memcpy(T, m->T, n * sizeof(double));
    return 0;
}

int orc_get_absorbed_sum(const orc_model* m, double* acc, size_t n)
{
    if (!m->acc || (int64_t)n != m->ncell) return -1;
    memcpy(acc, m->acc, n * sizeof(double));
    return 0;
}

int orc_get_absorbed_sum2(const orc_model* m, double* acc2, size_t n)
{
    if (!m->acc2 || (int64_t)n != m->ncell) return -1;
    memcpy(acc2, m->acc2, n * sizeof(double));
    return 0;
}

int orc_get_sed(const orc_model* m, double* sum, double* sum2, int64_t* count, size_t n)
{
    size_t ns = (size_t)m->n_incl * m->nnu;
    if (!m->sed_sum || n != ns) return -1;
    memcpy(sum, m->sed_sum, ns * sizeof(double));
    if (sum2) memcpy(sum2, m->sed_sum2, ns * sizeof(double));
    if (count) memcpy(count, m->sed_n, ns * sizeof(int64_t));
    return 0;
}

int orc_get_peeled_sed(const orc_model* m, double* sum, double* sum2, size_t n)
{
    size_t ns = (size_t)m->n_peel * 2 * m->nnu;
    if (n != ns) return -1;
    if (ns) {
        memcpy(sum, m->psed_sum, ns * sizeof(double));
        if (sum2) memcpy(sum2, m->psed_sum2, ns * sizeof(double));
    }
    return 0;
}

int orc_get_peeled_images(const orc_model* m, double* sum, double* sum2, size_t n)
{
    size_t ni = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    if (n != ni) return -1;
    if (ni) {
        memcpy(sum, m->pimg_sum, ni * sizeof(double));
        if (sum2) memcpy(sum2, m->pimg_sum2, ni * sizeof(double));
    }
    return 0;
}

int orc_get_images(const orc_model* m, double* sum, double* sum2, size_t n)
{
    size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    if (n != ni) return -1;
    if (ni == 0) return 0;
    memcpy(sum, m->img_sum, ni * sizeof(double));
    if (sum2) memcpy(sum2, m->img_sum2, ni * sizeof(double));
    return 0;
}

int orc_get_event_log(const orc_model* m, orc_event* ev, size_t cap, int32_t* counts, size_t n_counts)
{
    if (!m->evlog) return -1;
    size_t need = (size_t)m->ev_packets * m->ev_cap;
    if (cap < need || n_counts < (size_t)m->ev_packets) return -1;
    memcpy(ev, m->evlog, need * sizeof(orc_event));
    memcpy(counts, m->evcount, (size_t)m->ev_packets * sizeof(int32_t));
    return m->ev_packets;
}

int orc_get_emission_rows(const orc_model* m, int32_t* row, double* w, size_t n)
{
    if (!m->row_m || (int64_t)n != m->ncell) return -1;
    memcpy(row, m->row_m, n * sizeof(int32_t));
    memcpy(w, m->row_w, n * sizeof(double));
    return 0;
}

int64_t orc_trace_ray(const orc_model* m, const double x0[3], const double d[3], int64_t* cells,
                      double* lengths, int64_t cap)
{
    double x[3] = {x0[0], x0[1], x0[2]};
    int c[3];
    locate(m, x, d, c);
    int64_t n = 0;
    while (inside(m, c)) {
        double tw[3];
        for (int a = 0; a < 3; ++a) tw[a] = wall_distance(m, x, d, c, a);
        int ax = 0;
        if (tw[1] < tw[ax]) ax = 1;
        if (tw[2] < tw[ax]) ax = 2;
        double l = tw[ax] > 0.0 ? tw[ax] : 0.0;
        if (n >= cap) return -1;
        cells[n] = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
        lengths[n] = l;
        n++;
        for (int a = 0; a < 3; ++a) x[a] += d[a] * l;
        if (d[ax] > 0.0) {
            x[ax] = wall(m, ax, c[ax] + 1);
            c[ax] += 1;
        } else {
            x[ax] = wall(m, ax, c[ax]);
            c[ax] -= 1;
        }
    }
    return n;
}

/* ======================================================================= */
/* Raytracing of source and dust emission (Sec. 2.6.3).                    */
/* ======================================================================= */

/* Image axes of the observer direction o: e_x = norm(z x o) (e_x = x when o is
 * along z), e_y = o x e_x -- the axes of the peeled images. */
static void image_axes(const double o[3], double ex[3], double ey[3])
{
    ex[0] = -o[1];
    ex[1] = o[0];
    ex[2] = 0.0;
    double en = sqrt(ex[0] * ex[0] + ex[1] * ex[1]);
    if (en < 1e-12) {
        ex[0] = 1.0;
        ex[1] = 0.0;
    } else {
        ex[0] /= en;
        ex[1] /= en;
    }
    ey[0] = -o[2] * ex[1];
    ey[1] = o[2] * ex[0];
    ey[2] = o[0] * ex[1] - o[1] * ex[0];
}

/* The raytraced emission, in post-processing at the current temperatures,
 * toward every peel-off observer o.  The image has npix x npix pixels over
 * +-hw (cm) around the grid centre on the axes of image_axes.  Through each
 * pixel centre X e_x + Y e_y a ray is followed from the observer's side of
 * the grid along -o; in every bin k it accumulates the formal solution of the
 * transfer equation through cells of constant density and temperature,
 *     I_k = sum over cells, front to back, of
 *           exp(-tau_k in front of the cell) S_k (1 - exp(-dtau_k)),
 * with dtau_k = rho chi_k l over the cell's chord l and the source function
 * S_k = (kappa_k / chi_k) B_k(T): thermal emission rho kappa_k B_k(T) over
 * extinction rho chi_k, B_k the Planck function integrated over the bin (per
 * steradian).  Scattered light is not part of it (peeling-off's share).
 * cube[o][iy][ix][k] = I_k (2 hw / npix)^2 (erg/s/sr from the pixel); each
 * point source adds L_k / (4 pi) exp(-tau_k(source -> grid boundary along o))
 * to the pixel it projects into.  sed[o][0][k]: the sources, sed[o][1][k]: the
 * sum of the dust part over the pixels. */
int orc_raytrace(orc_model* m, int npix, double hw, double* cube, double* sed)
{
    if (!m->have_grid || !m->have_rho || !m->have_dust) return fail(m, "model is not set up");
    if (m->n_peel <= 0) return fail(m, "no observers: call orc_set_peeloff first");
    if (npix <= 0 || !(hw > 0.0)) return fail(m, "bad image size");
    const int nnu = m->nnu;
    const double apix = (2.0 * hw / npix) * (2.0 * hw / npix);
    double* I = (double*)malloc(2 * (size_t)nnu * sizeof(double));
    double* tau = I + nnu;
    double cen[3];
    for (int a = 0; a < 3; ++a) cen[a] = 0.5 * (m->lo[a] + m->hi[a]);
    memset(sed, 0, (size_t)m->n_peel * 2 * nnu * sizeof(double));
    for (int i = 0; i < m->n_peel; ++i) {
        const double* o = m->peel_dir + 3 * i;
        double ex[3], ey[3], d[3] = {-o[0], -o[1], -o[2]};
        image_axes(o, ex, ey);
        for (int iy = 0; iy < npix; ++iy)
            for (int ix = 0; ix < npix; ++ix) {
                double* out = cube + (((size_t)i * npix + iy) * npix + ix) * nnu;
                for (int k = 0; k < nnu; ++k) I[k] = tau[k] = 0.0;
                const double X = -hw + (ix + 0.5) * (2.0 * hw / npix);
                const double Y = -hw + (iy + 0.5) * (2.0 * hw / npix);
                double q[3];
                for (int a = 0; a < 3; ++a) q[a] = cen[a] + X * ex[a] + Y * ey[a];
                /* the line q + s o meets the grid box for s in [s0, s1] */
                double s0 = -INFINITY, s1 = INFINITY;
                int miss = 0;
                for (int a = 0; a < 3; ++a) {
                    if (o[a] != 0.0) {
                        double u = (m->lo[a] - q[a]) / o[a], v = (m->hi[a] - q[a]) / o[a];
                        if (u > v) { double w = u; u = v; v = w; }
                        if (u > s0) s0 = u;
                        if (v < s1) s1 = v;
                    } else if (q[a] < m->lo[a] || q[a] >= m->hi[a]) {
                        miss = 1;
                    }
                }
                if (!miss && s1 > s0) {
                    double x[3];
                    int c[3];
                    for (int a = 0; a < 3; ++a) x[a] = q[a] + s1 * o[a];
                    locate(m, x, d, c);
                    for (int a = 0; a < 3; ++a) { /* the entry point lies on the box */
                        if (c[a] < 0) c[a] = 0;
                        if (c[a] >= m->n[a]) c[a] = m->n[a] - 1;
                    }
                    while (inside(m, c)) {
                        double tw[3];
                        for (int a = 0; a < 3; ++a) tw[a] = wall_distance(m, x, d, c, a);
                        int ax = 0;
                        if (tw[1] < tw[ax]) ax = 1;
                        if (tw[2] < tw[ax]) ax = 2;
                        const double l = tw[ax] > 0.0 ? tw[ax] : 0.0;
                        const int64_t j = c[0] + (int64_t)m->n[0] * (c[1] + (int64_t)m->n[1] * c[2]);
                        const double r = m->rho[j];
                        if (r > 0.0) {
                            const double T = m->T[j];
                            for (int k = 0; k < nnu; ++k) {
                                const double dt = r * m->chi[k] * l;
                                const double S = T > 0.0 ? m->kap[k] / m->chi[k] *
                                                               orc_planck_bin(m->nu[k], m->nu[k + 1], T)
                                                         : 0.0;
                                I[k] += exp(-tau[k]) * S * -expm1(-dt);
                                tau[k] += dt;
                            }
                        }
                        for (int a = 0; a < 3; ++a) x[a] += d[a] * l;
                        if (d[ax] > 0.0) {
                            x[ax] = wall(m, ax, c[ax] + 1);
                            c[ax] += 1;
                        } else {
                            x[ax] = wall(m, ax, c[ax]);
                            c[ax] -= 1;
                        }
                    }
                }
                for (int k = 0; k < nnu; ++k) {
                    out[k] = I[k] * apix;
                    sed[((size_t)i * 2 + 1) * nnu + k] += out[k];
                }
            }
        /* point sources */
        for (int s = 0; s < m->nsrc; ++s) {
            const double* p = m->spos + 3 * s;
            double tot = 0.0;
            for (int k = 0; k < nnu; ++k) tot += m->sspec[(size_t)s * nnu + k];
            double pc[3];
            for (int a = 0; a < 3; ++a) pc[a] = p[a] - cen[a];
            const double X = pc[0] * ex[0] + pc[1] * ex[1] + pc[2] * ex[2];
            const double Y = pc[0] * ey[0] + pc[1] * ey[1] + pc[2] * ey[2];
            const double fx = floor((X + hw) / (2.0 * hw) * npix);
            const double fy = floor((Y + hw) / (2.0 * hw) * npix);
            const int in_img = fx >= 0.0 && fy >= 0.0 && fx < npix && fy < npix;
            for (int k = 0; k < nnu; ++k) {
                const double Lk = m->slum[s] * m->sspec[(size_t)s * nnu + k] / tot;
                const double v = Lk / (4.0 * ORC_PI) * exp(-tau_to_boundary(m, p, o, k));
                sed[((size_t)i * 2) * nnu + k] += v;
                if (in_img) cube[(((size_t)i * npix + (size_t)fy) * npix + (size_t)fx) * nnu + k] += v;
            }
        }
    }
    free(I);
    return 0;
}
