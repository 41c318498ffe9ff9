// mcrt_api.cpp -- host side of libmcrt: argument validation, FP64 table
// construction, device memory, and the Lucy iteration driver (Robitaille
// 2011, Sec. 2: inputs -> propagation -> Adot -> convergence -> SEDs/images).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>
#include <string>
#include <type_traits>
#include <vector>

#include "mcrt_internal.h"
#include "mcrt_tables.h"

namespace mcrt {
template <typename R>
hipError_t launch_transport(const TransportParams<R>& P, int K, int brick, int blocks, int threads,
                            hipStream_t st);
template <typename R> int transport_max_blocks_per_cu(int K, int brick, int threads, size_t lds);
template <typename R> size_t transport_lds_bytes(const TransportParams<R>& P);
hipError_t launch_to_bricks_f32(int64_t n, int nx, int ny, int bx, int bxy, const float* in,
                                float* out, int blocks, hipStream_t st);
hipError_t launch_to_bricks_f64(int64_t n, int nx, int ny, int bx, int bxy, const double* in,
                                double* out, int blocks, hipStream_t st);
hipError_t launch_rows64(int64_t, const double*, const double*, double*, unsigned long long*, int,
                         hipStream_t);
hipError_t launch_rows32(int64_t, const double*, const double*, float*, unsigned long long*, int,
                         hipStream_t);
hipError_t launch_update(const CellParams& P, int blocks, hipStream_t st);
hipError_t launch_select(int64_t n, const double* v, unsigned long long* sel, unsigned int* hist,
                         int blocks, hipStream_t st);
hipError_t launch_to_f32(int64_t n, const double* in, float* out, int blocks, hipStream_t st);
hipError_t launch_to_f64(int64_t n, const float* in, double* out, int blocks, hipStream_t st);
hipError_t launch_check_T(int64_t n, const double* T, unsigned long long* bad, int blocks,
                          hipStream_t st);
hipError_t launch_check_rho(int64_t n, const double* rho, unsigned long long* bad, int blocks,
                            hipStream_t st);
hipError_t launch_fill_u8(int64_t n, unsigned char* p, unsigned char v, int blocks, hipStream_t st);
hipError_t launch_fill_f64(int64_t n, double* p, double v, int blocks, hipStream_t st);
hipError_t launch_fill_u64(int64_t n, unsigned long long* p, unsigned long long v, int blocks,
                           hipStream_t st);
size_t sweep_record_bytes(int fp32);
template <typename R>
hipError_t launch_sweep_step(const TransportParams<R>& P, const SweepParams& S, int b, bool full,
                             int emit_blocks, int group_blocks, int blocks, int threads, size_t lds,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1);
template <typename R>
hipError_t launch_sweep_drain(const TransportParams<R>& P, const SweepParams& S, int b, int blocks,
                              hipStream_t st);
template <typename R> hipError_t sweep_prepare(bool noise, bool full, size_t lds);
template <typename R> int sweep_max_blocks_per_cu(bool noise, bool full, int threads, size_t lds);
int sweep_emit_step();
hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st);
hipError_t launch_rotate(int fp32, const double* d, const double* mu, const double* phi, double* out,
                         int n, hipStream_t st);
hipError_t launch_raytrace(const RayParams& R, hipStream_t st);
hipError_t launch_pda_coefficients(const PdaParams& P, int select, hipStream_t st);
hipError_t launch_pda_connect(const PdaParams& P, hipStream_t st);
hipError_t launch_pda_init(const PdaParams& P, hipStream_t st);
hipError_t launch_pda_iteration(const PdaParams& P, hipStream_t st);
hipError_t launch_pda_shift(const PdaParams& P, hipStream_t st);
hipError_t launch_pda_finish(const PdaParams& P, hipStream_t st);
}  // namespace mcrt

using namespace mcrt;

namespace {

template <typename T> struct DBuf {
    T* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t count) {
        if (count <= n && p) return hipSuccess;
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
        hipError_t e = hipMalloc((void**)&p, (count ? count : 1) * sizeof(T));
        if (e == hipSuccess) n = count;
        return e;
    }
    void release() {
        if (p) hipFree(p);
        p = nullptr;
        n = 0;
    }
};

// Device memory of the tiled sweeps' record and entry buffers (tens of GB for
// a pass of 1e8 packets).  Blocks a model lets go of stay with the process,
// per device, and serve the next model that needs at most their size, so a
// series of models (a warm-start comparison, a test suite) does not map and
// unmap that memory once per model.  When the device runs out of memory the
// device's idle blocks are freed and the allocation is tried again.
struct PoolBlock {
    int device;
    void* p;
    size_t bytes;
};
std::mutex g_pool_mu;
std::vector<PoolBlock> g_pool;

hipError_t pool_get(int device, size_t bytes, void** out, size_t* got) {
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        size_t best = g_pool.size();
        for (size_t i = 0; i < g_pool.size(); ++i)
            if (g_pool[i].device == device && g_pool[i].bytes >= bytes &&
                (best == g_pool.size() || g_pool[i].bytes < g_pool[best].bytes))
                best = i;
        if (best < g_pool.size()) {
            *out = g_pool[best].p;
            *got = g_pool[best].bytes;
            g_pool.erase(g_pool.begin() + (std::ptrdiff_t)best);
            return hipSuccess;
        }
    }
    hipError_t e = hipMalloc(out, bytes);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            for (size_t i = 0; i < g_pool.size();) {
                if (g_pool[i].device == device) {
                    hipFree(g_pool[i].p);
                    g_pool.erase(g_pool.begin() + (std::ptrdiff_t)i);
                } else {
                    ++i;
                }
            }
        }
        e = hipMalloc(out, bytes);
    }
    *got = e == hipSuccess ? bytes : 0;
    return e;
}

void pool_put(int device, void* p, size_t bytes) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    g_pool.push_back(PoolBlock{device, p, bytes});
}

template <typename T> struct PoolBuf {
    T* p = nullptr;
    size_t n = 0;
    size_t bytes = 0;
    int device = 0;
    hipError_t ensure(int dev, size_t count) {
        if (count <= n && p) return hipSuccess;
        release();
        void* q = nullptr;
        size_t got = 0;
        const hipError_t e = pool_get(dev, (count ? count : 1) * sizeof(T), &q, &got);
        if (e == hipSuccess) {
            p = static_cast<T*>(q);
            n = got / sizeof(T);
            bytes = got;
            device = dev;
        }
        return e;
    }
    void release() {
        if (p) pool_put(device, p, bytes);
        p = nullptr;
        n = 0;
        bytes = 0;
    }
};

struct Source {
    double pos[3];
    double lum;
    std::vector<double> spec;  // relative luminosity per bin
};

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

}  // namespace

struct mcrt_model {
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int n_cu = 256;
    size_t mem_total = 0;  // device memory, bytes
    // problem
    bool have_grid = false, have_rho = false, have_nu = false, have_dust = false,
         have_obs = false, have_run = false;
    int n[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0}, dx[3] = {0, 0, 0}, vol = 0.0;
    int64_t ncell = 0;
    std::vector<double> nu, chi, alb, g, kap;
    std::vector<Source> src;
    int n_incl = 10, npix = 0, n_img = 0;
    double img_hw = 0.0;
    std::vector<int> img_bins;
    mcrt_run_cfg cfg;
    bool tables_dirty = true;
    bool state_ready = false;
    // device problem data
    DBuf<double> rho64;
    DBuf<float> rho32;
    DBuf<double> chi64, kap64, alb64, g64, lcdf64, scdf64, ecdf64;
    DBuf<float> chi32, kap32, alb32, g32, lcdf32, scdf32, ecdf32;
    DBuf<double> spos, sweight, lnA, slope;
    DBuf<int4> scell;
    DBuf<double> sfrac;
    DBuf<double> ecoarse64, scoarse64;
    DBuf<float> ecoarse32, scoarse32;
    int npad = 0, ngroup = 0;
    // density in the transport layout: x-fastest (aliases rho64/rho32) or bricks
    DBuf<double> rhoT64;
    DBuf<float> rhoT32;
    int t_layout = -1;      // layout the transport density arrays hold, -1 = none yet
    int bx = 0, by = 0, bz = 0;
    int64_t nt_cells = 0;   // length of the transport-layout arrays
    size_t acc_stride = 0;  // elements per tally copy
    int acc_copies = 1;     // tally copies of the last transport
    DBuf<int> img_of_bin;
    double dy = 0.0;
    double ltot = 0.0;
    // device state
    DBuf<double> acc, acc2, adot, adot_prev, adot_sig, T, T_prev, sig_rel, sig_rel_prev;
    DBuf<unsigned char> valid, valid_prev;
    DBuf<double> rowpos64, Rbuf, rbuf;
    DBuf<float> rowpos32;
    DBuf<double> sed_sum, sed_sum2, img_sum, img_sum2;
    int n_peel = 0;
    DBuf<double> peel_dir, psed_sum, psed_sum2, pimg_sum, pimg_sum2;
    // raytracing: spectral cube and SED of the last mcrt_raytrace, its image
    DBuf<double> ray_cube, ray_sed, ray_nu, ray_lsrc;
    DBuf<double> ray_btab;          // raytracing table of ln B_k(ln T), built on first use
    bool ray_btab_ok = false;
    // modified random walk: Planck/Rosseland mean table (built when mrw_gamma > 0
    // or for the partial diffusion approximation)
    DBuf<double> mrw_tab;
    DBuf<double> mrw_ytab;          // the walk's first-passage inverse (the same for every model)
    bool mrw_tab_built = false;
    // partial diffusion approximation: flags, CG vectors (8 x ncell), reductions
    DBuf<unsigned char> pda_flag;
    DBuf<double> pda_vec, pda_red;
    DBuf<unsigned> pda_count;
    int ray_npix = 0;
    DBuf<unsigned long long> sed_n;
    DBuf<mcrt_event> evlog;
    DBuf<int32_t> evcount;
    DBuf<unsigned long long> misc;  // pool, counters[C_COUNT], stats[8], sel[3], scratch
    DBuf<double> energies;
    DBuf<unsigned int> hist;
    // tiled sweeps: packet records (two buffers), registered entries (two
    // lists), entries grouped by tile, per-tile counts, offsets and cursors,
    // control words; pinned host copies of the termination flag and events
    // for the lagged check of the host loop
    PoolBuf<uint4> sw_rec[2];
    PoolBuf<unsigned> sw_ent_tile[2];
    PoolBuf<uint2> sw_ent[2], sw_sent;
    DBuf<unsigned> sw_tile_rec, sw_tile_ent, sw_ent_off, sw_cursor;
    DBuf<uint4> sw_item_desc;
    DBuf<SweepCtl> sw_ctl;
    unsigned* sw_host = nullptr;   // [kSweepLag] done flags
    hipEvent_t sw_ev[4] = {nullptr, nullptr, nullptr, nullptr};
    std::vector<hipEvent_t> sw_kev;  // pairs bracketing each sweep kernel of a pass
    size_t lds_max = 65536 - 1024;  // dynamic LDS a transport kernel may take
    int64_t ev_packets = 0;
    int ev_cap = 0;
    // iteration state
    int iter = 0;
    int have_prev = 0;
    double q_prev = INFINITY;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

constexpr int kMaxTallyCopies = 8;  // one per XCD of an MI355X
constexpr int MISC_POOL = 0;
constexpr int MISC_CNT = 1;                  // C_COUNT entries
constexpr int MISC_STATS = 1 + C_COUNT;      // 8 entries
constexpr int MISC_SEL = MISC_STATS + 8;     // 3 entries
constexpr int MISC_SCRATCH = MISC_SEL + 3;   // 2 entries
constexpr int MISC_N = MISC_SCRATCH + 2;

mcrt_status fail(mcrt_model* m, mcrt_status s, const std::string& msg) {
    m->err = msg;
    return s;
}

// Staging of mcrt_scatter_directions_noalloc: per direction its input vector,
// mu, phi and output vector (9 doubles), for at most kNoAllocDirs directions
// (4.5 MiB).  Every GPU the library runs on holds its own copy until the
// process ends.  In host code the array's name is not a device address: the
// address each device's copy has is looked up once per device, with that
// device current, and kept in g_scratch_ptr.
constexpr int kNoAllocDirs = 1 << 16;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[9 * kNoAllocDirs];
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_setup(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[dev]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) g_scratch_ptr[dev] = static_cast<double*>(p);
    if (cur != dev) hipSetDevice(cur);
    return e != hipSuccess ? e : (p ? hipSuccess : hipErrorInvalidSymbol);
}

double* scratch_ptr(int dev) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return dev >= 0 && dev < kMaxDevices ? g_scratch_ptr[dev] : nullptr;
}

#define HIPCHK(expr)                                                                         \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(m, e_ == hipErrorOutOfMemory ? MCRT_E_NOMEM : MCRT_E_DEVICE,         \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

int grid_blocks(const mcrt_model* m, int64_t n) {
    int64_t b = (n + 255) / 256;
    int64_t cap = (int64_t)m->n_cu * 8;
    if (b > cap) b = cap;
    return (int)(b < 1 ? 1 : b);
}

template <typename T>
hipError_t upload(DBuf<T>& b, const std::vector<T>& h, hipStream_t st) {
    hipError_t e = b.ensure(h.size());
    if (e != hipSuccess) return e;
    if (h.empty()) return hipSuccess;
    return hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, st);
}

std::vector<float> to_f32(const std::vector<double>& v) {
    return std::vector<float>(v.begin(), v.end());
}

// Rows of nb CDF values padded to npad = kGroup*ngroup entries with 2.0 (never
// selected: uniforms are < 1 = the last real entry), and the coarse index of
// every group's last entry for the two-level search of the transport kernel.
void pad_rows(const std::vector<double>& rows, size_t nrow, size_t nb, size_t npad, size_t ng,
              std::vector<double>& padded, std::vector<double>& coarse) {
    padded.assign(nrow * npad, 2.0);
    coarse.assign(nrow * ng, 2.0);
    for (size_t r = 0; r < nrow; ++r) {
        for (size_t k = 0; k < nb; ++k) padded[r * npad + k] = rows[r * nb + k];
        for (size_t q = 0; q < ng; ++q) coarse[r * ng + q] = padded[r * npad + kGroup * q + kGroup - 1];
    }
}

// The emissivity rows and the T-solve table depend on the frequency edges and
// kappa alone and take most of a model's set-up time (thousands of Planck bin
// integrals); the last few sets built in the process are kept and reused for
// models with identical frequency edges and kappa (a family of models sharing
// one dust, set up one after another).
struct DustTables {
    std::vector<double> nu, kap, ecdf, lnA, slope;
    double dy = 0.0;
};
std::mutex g_dust_mu;
std::vector<DustTables> g_dust;  // most recent last
constexpr size_t kDustCache = 4;

void dust_tables(const std::vector<double>& nu, const std::vector<double>& kap, std::vector<double>& ecdf,
                 std::vector<double>& lnA, std::vector<double>& slope, double* dy) {
    {
        std::lock_guard<std::mutex> lk(g_dust_mu);
        for (size_t i = 0; i < g_dust.size(); ++i) {
            if (g_dust[i].nu == nu && g_dust[i].kap == kap) {
                ecdf = g_dust[i].ecdf;
                lnA = g_dust[i].lnA;
                slope = g_dust[i].slope;
                *dy = g_dust[i].dy;
                return;
            }
        }
    }
    DustTables t;
    t.nu = nu;
    t.kap = kap;
    emission_rows(nu, kap, t.ecdf);
    tsolve_table(nu, kap, t.lnA, t.slope, &t.dy);
    ecdf = t.ecdf;
    lnA = t.lnA;
    slope = t.slope;
    *dy = t.dy;
    std::lock_guard<std::mutex> lk(g_dust_mu);
    if (g_dust.size() == kDustCache) g_dust.erase(g_dust.begin());
    g_dust.push_back(std::move(t));
}

// The raytracing table of ln B_k(ln T) depends on the frequency edges alone;
// the last few built in the process are reused.
std::mutex g_btab_mu;
std::vector<std::pair<std::vector<double>, std::vector<double>>> g_btab;  // (nu, table), most recent last

void ray_planck_table(const std::vector<double>& nu, std::vector<double>& tab) {
    {
        std::lock_guard<std::mutex> lk(g_btab_mu);
        for (const auto& e : g_btab)
            if (e.first == nu) {
                tab = e.second;
                return;
            }
    }
    planck_ln_table(nu, tab);
    std::lock_guard<std::mutex> lk(g_btab_mu);
    if (g_btab.size() == kDustCache) g_btab.erase(g_btab.begin());
    g_btab.emplace_back(nu, tab);
}

// The Planck- and Rosseland-mean table of the modified random walk and the
// diffusion approximation depends on the frequency edges, kappa and chi; the
// last few built in the process are reused.
struct MeanTables {
    std::vector<double> nu, kap, chi, tab;
};
std::mutex g_mean_mu;
std::vector<MeanTables> g_mean;  // most recent last

void mean_opacity_table(const std::vector<double>& nu, const std::vector<double>& kap,
                        const std::vector<double>& chi, std::vector<double>& tab) {
    {
        std::lock_guard<std::mutex> lk(g_mean_mu);
        for (const MeanTables& e : g_mean)
            if (e.nu == nu && e.kap == kap && e.chi == chi) {
                tab = e.tab;
                return;
            }
    }
    mrw_table(nu, kap, chi, tab);
    std::lock_guard<std::mutex> lk(g_mean_mu);
    if (g_mean.size() == kDustCache) g_mean.erase(g_mean.begin());
    g_mean.push_back(MeanTables{nu, kap, chi, tab});
}

// The walk's first-passage inverse depends on nothing of a model: built once
// per process.
const std::vector<double>& escape_table() {
    static std::once_flag once;
    static std::vector<double> tab;
    std::call_once(once, [] { mrw_escape_table(tab); });
    return tab;
}

mcrt_status build_tables(mcrt_model* m) {
    m->ray_btab_ok = false;
    const size_t nb = m->kap.size();
    const size_t ns = m->src.size();
    const size_t ng = (nb + kGroup - 1) / kGroup, npad = ng * kGroup;
    m->ngroup = (int)ng;
    m->npad = (int)npad;
    // sources: spectral CDFs, luminosity CDF
    std::vector<double> scdf(ns * nb), lcdf(ns), spos(3 * ns);
    m->ltot = 0.0;
    for (const Source& s : m->src) m->ltot += s.lum;
    double acc = 0.0;
    std::vector<double> c;
    for (size_t i = 0; i < ns; ++i) {
        cumulative(m->src[i].spec, c);
        for (size_t k = 0; k < nb; ++k) scdf[i * nb + k] = c[k];
        acc += m->src[i].lum;
        lcdf[i] = acc / m->ltot;
        for (int a = 0; a < 3; ++a) spos[3 * i + a] = m->src[i].pos[a];
    }
    // each source's cell, from the same FP64 arithmetic as the emission's
    std::vector<int4> scell(ns);
    std::vector<double> sfrac(3 * ns);
    for (size_t i = 0; i < ns; ++i) {
        int c[3], w = 0;
        for (int a = 0; a < 3; ++a) {
            const double fp = (m->src[i].pos[a] - m->lo[a]) / m->dx[a];
            const double fl = std::floor(fp);
            c[a] = (int)fl;
            sfrac[3 * i + a] = fp - fl;
            if (fp == fl) w |= 1 << a;
        }
        scell[i] = make_int4(c[0], c[1], c[2], w);
    }
    lcdf.back() = 1.0;
    std::vector<double> ecdf, lnA, slope;
    dust_tables(m->nu, m->kap, ecdf, lnA, slope, &m->dy);
    std::vector<double> scdf_p, scoarse, ecdf_p, ecoarse;
    pad_rows(scdf, ns, nb, npad, ng, scdf_p, scoarse);
    pad_rows(ecdf, kRows, nb, npad, ng, ecdf_p, ecoarse);
    std::vector<int> iob(nb, -1);
    for (int i = 0; i < m->n_img; ++i) iob[m->img_bins[i]] = i;
    hipStream_t st = m->stream;
    HIPCHK(upload(m->chi64, m->chi, st));
    HIPCHK(upload(m->kap64, m->kap, st));
    HIPCHK(upload(m->alb64, m->alb, st));
    HIPCHK(upload(m->g64, m->g, st));
    HIPCHK(upload(m->lcdf64, lcdf, st));
    HIPCHK(upload(m->scdf64, scdf_p, st));
    HIPCHK(upload(m->ecdf64, ecdf_p, st));
    HIPCHK(upload(m->scoarse64, scoarse, st));
    HIPCHK(upload(m->ecoarse64, ecoarse, st));
    // host copies stay alive until the stream synchronisation below
    const std::vector<float> chi32 = to_f32(m->chi), kap32 = to_f32(m->kap),
                             alb32 = to_f32(m->alb), g32 = to_f32(m->g);
    HIPCHK(upload(m->chi32, chi32, st));
    HIPCHK(upload(m->kap32, kap32, st));
    HIPCHK(upload(m->alb32, alb32, st));
    HIPCHK(upload(m->g32, g32, st));
    std::vector<float> lcdf32 = to_f32(lcdf), scdf32 = to_f32(scdf_p), ecdf32 = to_f32(ecdf_p);
    // a rounded CDF must still end at exactly 1
    lcdf32.back() = 1.0f;
    for (size_t i = 0; i < ns; ++i) scdf32[i * npad + nb - 1] = 1.0f;
    for (int r = 0; r < kRows; ++r) ecdf32[(size_t)r * npad + nb - 1] = 1.0f;
    std::vector<float> scoarse32(ns * ng), ecoarse32((size_t)kRows * ng);
    for (size_t r = 0; r < ns; ++r)
        for (size_t q = 0; q < ng; ++q) scoarse32[r * ng + q] = scdf32[r * npad + kGroup * q + kGroup - 1];
    for (size_t r = 0; r < (size_t)kRows; ++r)
        for (size_t q = 0; q < ng; ++q) ecoarse32[r * ng + q] = ecdf32[r * npad + kGroup * q + kGroup - 1];
    HIPCHK(upload(m->lcdf32, lcdf32, st));
    HIPCHK(upload(m->scdf32, scdf32, st));
    HIPCHK(upload(m->ecdf32, ecdf32, st));
    HIPCHK(upload(m->scoarse32, scoarse32, st));
    HIPCHK(upload(m->ecoarse32, ecoarse32, st));
    HIPCHK(upload(m->spos, spos, st));
    HIPCHK(upload(m->scell, scell, st));
    HIPCHK(upload(m->sfrac, sfrac, st));
    HIPCHK(upload(m->lnA, lnA, st));
    HIPCHK(upload(m->slope, slope, st));
    HIPCHK(upload(m->img_of_bin, iob, st));
    std::vector<double> mrw;
    if (m->cfg.mrw_gamma > 0.0) {
        mean_opacity_table(m->nu, m->kap, m->chi, mrw);
        HIPCHK(upload(m->mrw_tab, mrw, st));
        HIPCHK(upload(m->mrw_ytab, escape_table(), st));
    }
    m->mrw_tab_built = m->cfg.mrw_gamma > 0.0;
    HIPCHK(hipStreamSynchronize(st));
    m->tables_dirty = false;
    return MCRT_OK;
}

// Density arrays in the transport layout (x-fastest or 4x4x4 bricks).
mcrt_status ensure_transport_grid(mcrt_model* m, int layout) {
    m->bx = (m->n[0] + 3) / 4;
    m->by = (m->n[1] + 3) / 4;
    m->bz = (m->n[2] + 3) / 4;
    if (m->t_layout == layout) return MCRT_OK;
    hipStream_t st = m->stream;
    const int b = grid_blocks(m, m->ncell);
    if (layout == 1) {
        const int64_t nt = (int64_t)m->bx * m->by * m->bz * 64;
        HIPCHK(m->rhoT64.ensure(nt));
        HIPCHK(m->rhoT32.ensure(nt));
        HIPCHK(hipMemsetAsync(m->rhoT64.p, 0, nt * sizeof(double), st));
        HIPCHK(hipMemsetAsync(m->rhoT32.p, 0, nt * sizeof(float), st));
        HIPCHK(launch_to_bricks_f64(m->ncell, m->n[0], m->n[1], m->bx, m->bx * m->by, m->rho64.p,
                                    m->rhoT64.p, b, st));
        HIPCHK(launch_to_bricks_f32(m->ncell, m->n[0], m->n[1], m->bx, m->bx * m->by, m->rho32.p,
                                    m->rhoT32.p, b, st));
        m->nt_cells = nt;
    } else {
        m->rhoT64.release();
        m->rhoT32.release();
        m->nt_cells = m->ncell;
    }
    HIPCHK(hipStreamSynchronize(st));
    m->t_layout = layout;
    return MCRT_OK;
}

mcrt_status ensure_state(mcrt_model* m) {
    if (m->state_ready) return MCRT_OK;
    const size_t nc = (size_t)m->ncell;
    // tallies are indexed in the transport layout; bricks pad each axis to 4
    const size_t nbrick = (size_t)((m->n[0] + 3) / 4) * ((m->n[1] + 3) / 4) * ((m->n[2] + 3) / 4) * 64;
    m->acc_stride = nbrick > nc ? nbrick : nc;
    HIPCHK(m->acc.ensure(kMaxTallyCopies * m->acc_stride));
    HIPCHK(m->acc2.ensure(m->acc_stride));
    HIPCHK(m->adot.ensure(nc));
    HIPCHK(m->adot_prev.ensure(nc));
    HIPCHK(m->adot_sig.ensure(nc));
    HIPCHK(m->T.ensure(nc));
    HIPCHK(m->T_prev.ensure(nc));
    HIPCHK(m->sig_rel.ensure(nc));
    HIPCHK(m->sig_rel_prev.ensure(nc));
    HIPCHK(m->valid.ensure(nc));
    HIPCHK(m->valid_prev.ensure(nc));
    HIPCHK(m->Rbuf.ensure(nc));
    HIPCHK(m->rbuf.ensure(nc));
    HIPCHK(m->misc.ensure(MISC_N));
    HIPCHK(m->energies.ensure(2));
    HIPCHK(m->hist.ensure(256));
    hipStream_t st = m->stream;
    const int b = grid_blocks(m, m->ncell);
    HIPCHK(launch_fill_f64(m->ncell, m->T.p, m->cfg.t_init, b, st));
    HIPCHK(launch_fill_f64(m->ncell, m->adot.p, 0.0, b, st));
    HIPCHK(launch_fill_f64(m->ncell, m->sig_rel.p, 0.0, b, st));
    HIPCHK(launch_fill_f64(m->ncell, m->adot_sig.p, 0.0, b, st));
    HIPCHK(launch_fill_u8(m->ncell, m->valid.p, 1, b, st));
    HIPCHK(hipMemsetAsync(m->hist.p, 0, 256 * sizeof(unsigned int), st));
    HIPCHK(hipStreamSynchronize(st));
    m->iter = 0;
    m->have_prev = 0;
    m->q_prev = INFINITY;
    m->state_ready = true;
    return MCRT_OK;
}

mcrt_status ensure_bins(mcrt_model* m) {
    const size_t ns = (size_t)m->n_incl * m->kap.size();
    const size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    HIPCHK(m->sed_sum.ensure(ns));
    HIPCHK(m->sed_sum2.ensure(ns));
    HIPCHK(m->sed_n.ensure(ns));
    HIPCHK(m->img_sum.ensure(ni));
    HIPCHK(m->img_sum2.ensure(ni));
    const size_t nps = (size_t)m->n_peel * 2 * m->kap.size();
    const size_t npi = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    HIPCHK(m->psed_sum.ensure(nps));
    HIPCHK(m->psed_sum2.ensure(nps));
    HIPCHK(m->pimg_sum.ensure(npi));
    HIPCHK(m->pimg_sum2.ensure(npi));
    return MCRT_OK;
}

mcrt_status clear_bins(mcrt_model* m) {
    const size_t ns = (size_t)m->n_incl * m->kap.size();
    const size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    hipStream_t st = m->stream;
    HIPCHK(hipMemsetAsync(m->sed_sum.p, 0, ns * sizeof(double), st));
    HIPCHK(hipMemsetAsync(m->sed_sum2.p, 0, ns * sizeof(double), st));
    HIPCHK(hipMemsetAsync(m->sed_n.p, 0, ns * sizeof(unsigned long long), st));
    if (ni) {
        HIPCHK(hipMemsetAsync(m->img_sum.p, 0, ni * sizeof(double), st));
        HIPCHK(hipMemsetAsync(m->img_sum2.p, 0, ni * sizeof(double), st));
    }
    const size_t nps = (size_t)m->n_peel * 2 * m->kap.size();
    const size_t npi = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    if (nps) {
        HIPCHK(hipMemsetAsync(m->psed_sum.p, 0, nps * sizeof(double), st));
        HIPCHK(hipMemsetAsync(m->psed_sum2.p, 0, nps * sizeof(double), st));
    }
    if (npi) {
        HIPCHK(hipMemsetAsync(m->pimg_sum.p, 0, npi * sizeof(double), st));
        HIPCHK(hipMemsetAsync(m->pimg_sum2.p, 0, npi * sizeof(double), st));
    }
    return MCRT_OK;
}

mcrt_status ready(mcrt_model* m) {
    if (!m->have_grid || !m->have_rho) return fail(m, MCRT_E_STATE, "grid and density must be set");
    if (!m->have_dust) return fail(m, MCRT_E_STATE, "dust must be set");
    if (m->src.empty()) return fail(m, MCRT_E_STATE, "add at least one source");
    if (!m->have_run) return fail(m, MCRT_E_STATE, "run parameters must be set");
    if (!m->have_obs) {
        mcrt_status s = mcrt_set_observers(m, 10, 0, 0.0, nullptr, 0);
        if (s != MCRT_OK) return s;
    }
    if (m->tables_dirty) {
        mcrt_status s = build_tables(m);
        if (s != MCRT_OK) return s;
    }
    mcrt_status s = ensure_state(m);
    if (s != MCRT_OK) return s;
    return ensure_bins(m);
}

// Equal-number sampling weights of a pass of np packets: source i gets
// floor(np/ns) or one more packets, each carrying L_i / count (relative to eps0).
mcrt_status set_weights(mcrt_model* m, int64_t np) {
    const double eps0 = m->ltot / (double)np;
    const size_t ns = m->src.size();
    std::vector<double> sw(ns);
    for (size_t i = 0; i < ns; ++i) {
        const int64_t cnt = np / (int64_t)ns + ((int64_t)i < np % (int64_t)ns ? 1 : 0);
        sw[i] = (m->src[i].lum / (double)(cnt > 0 ? cnt : 1)) / eps0;
    }
    HIPCHK(m->sweight.ensure(ns));
    HIPCHK(hipMemcpy(m->sweight.p, sw.data(), ns * sizeof(double), hipMemcpyHostToDevice));
    return MCRT_OK;
}

// Device work before a transport pass: emission rows from T, zeroed tallies and
// counters, event-log buffers.  graph_safe clears with fill kernels (a captured
// graph records no memset nodes).
mcrt_status prepare_pass(mcrt_model* m, int64_t np, bool graph_safe, bool per_lane) {
    hipStream_t s = m->stream;
    const size_t nc = (size_t)m->ncell;
    const bool f32 = m->cfg.precision == MCRT_FP32_TRANSPORT;
    unsigned long long* misc = m->misc.p;
    // the per-lane walk (transport_mode 0, and every batched launch) reads the
    // grid in the model's layout and adds into per-XCD tally copies; the tiled
    // sweeps read x-fastest and flush into one copy
    const int layout = m->cfg.grid_layout == 1 && per_lane ? 1 : 0;
    {
        mcrt_status r = ensure_transport_grid(m, layout);
        if (r != MCRT_OK) return r;
    }
    if (f32) HIPCHK(m->rowpos32.ensure(nc));
    else HIPCHK(m->rowpos64.ensure(nc));
    const size_t nt = (size_t)m->nt_cells;
    m->acc_copies = m->cfg.tally_copies == kMaxTallyCopies && per_lane ? kMaxTallyCopies : 1;
    const size_t nacc = (m->acc_copies - 1) * m->acc_stride + nt;
    m->ev_packets = m->cfg.event_log_packets < np ? m->cfg.event_log_packets : np;
    m->ev_cap = m->cfg.event_log_cap > 0 ? m->cfg.event_log_cap : 256;
    if (m->ev_packets > 0) {
        HIPCHK(m->evlog.ensure((size_t)m->ev_packets * m->ev_cap));
        HIPCHK(m->evcount.ensure((size_t)m->ev_packets));
    }
    if (graph_safe) {
        HIPCHK(launch_fill_u64(MISC_N, misc, 0ull, 1, s));
        HIPCHK(launch_fill_f64(2, m->energies.p, 0.0, 1, s));
        HIPCHK(launch_fill_f64((int64_t)nacc, m->acc.p, 0.0, grid_blocks(m, (int64_t)nacc), s));
        if (m->cfg.want_noise)
            HIPCHK(launch_fill_f64((int64_t)nt, m->acc2.p, 0.0, grid_blocks(m, (int64_t)nt), s));
        if (m->ev_packets > 0)
            HIPCHK(launch_fill_u8((int64_t)m->ev_packets * 4, (unsigned char*)m->evcount.p, 0,
                                  grid_blocks(m, m->ev_packets), s));
    } else {
        HIPCHK(hipMemsetAsync(misc, 0, MISC_N * sizeof(unsigned long long), s));
        HIPCHK(hipMemsetAsync(m->energies.p, 0, 2 * sizeof(double), s));
        HIPCHK(hipMemsetAsync(m->acc.p, 0, nacc * sizeof(double), s));
        if (m->cfg.want_noise) HIPCHK(hipMemsetAsync(m->acc2.p, 0, nt * sizeof(double), s));
        if (m->ev_packets > 0)
            HIPCHK(hipMemsetAsync(m->evcount.p, 0, (size_t)m->ev_packets * sizeof(int32_t), s));
    }
    const int cb = grid_blocks(m, m->ncell);
    if (f32)
        HIPCHK(launch_rows32(m->ncell, m->T.p, m->rho64.p, m->rowpos32.p, misc + MISC_SCRATCH, cb, s));
    else
        HIPCHK(launch_rows64(m->ncell, m->T.p, m->rho64.p, m->rowpos64.p, misc + MISC_SCRATCH, cb, s));
    return MCRT_OK;
}

int walk_batch_of(const mcrt_model* m) {
    const int w = m->cfg.walk_batch;
    return w == 1 || w == 2 || w == 8 ? w : 4;
}

// Launch parameters of one model's pass (prepare_pass must have run).
template <typename R>
void make_params(mcrt_model* m, int64_t np, uint32_t key1, int binning, TransportParams<R>& P) {
    constexpr bool f32 = std::is_same<R, float>::value;
    const int layout = m->t_layout == 1 ? 1 : 0;
    unsigned long long* misc = m->misc.p;
    // coarse CDF indices and the luminosity CDF go to LDS when they are small
    const size_t lds_need = (size_t)(m->src.size() + (kRows + m->src.size()) * m->ngroup) * sizeof(R);
    const int lds_tables = lds_need <= 32768 ? 1 : 0;
    const double eps0 = m->ltot / (double)np;
    P = TransportParams<R>{};
    const R *rho, *chi, *kap, *alb, *gg, *lcdf, *scdf, *ecdf, *rowpos, *scoarse, *ecoarse;
    if constexpr (f32) {
        rho = layout ? m->rhoT32.p : m->rho32.p;
        chi = m->chi32.p; kap = m->kap32.p; alb = m->alb32.p; gg = m->g32.p;
        lcdf = m->lcdf32.p; scdf = m->scdf32.p; ecdf = m->ecdf32.p; rowpos = m->rowpos32.p;
        scoarse = m->scoarse32.p; ecoarse = m->ecoarse32.p;
    } else {
        rho = layout ? m->rhoT64.p : m->rho64.p;
        chi = m->chi64.p; kap = m->kap64.p; alb = m->alb64.p; gg = m->g64.p;
        lcdf = m->lcdf64.p; scdf = m->scdf64.p; ecdf = m->ecdf64.p; rowpos = m->rowpos64.p;
        scoarse = m->scoarse64.p; ecoarse = m->ecoarse64.p;
    }
    {
        for (int a = 0; a < 3; ++a) {
            P.n[a] = m->n[a];
            P.lo[a] = m->lo[a];
            P.dx[a] = m->dx[a];
            P.dxr[a] = (R)m->dx[a];
            P.inv_dx[a] = (R)(1.0 / m->dx[a]);
        }
        P.bx = m->bx;
        P.bxy = m->bx * m->by;
        P.rho = rho;
        P.npad = m->npad;
        P.ngroup = m->ngroup;
        P.scoarse = scoarse;
        P.ecoarse = ecoarse;
        P.lds_tables = lds_tables;
        P.nnu = (int)m->kap.size();
        P.chi = chi;
        P.kap = kap;
        P.alb = alb;
        P.g = gg;
        P.nsrc = (int)m->src.size();
        P.sampling = m->cfg.source_sampling;
        P.spos = m->spos.p;
        P.scell = m->scell.p;
        P.sfrac = m->sfrac.p;
        P.lcdf = lcdf;
        P.scdf = scdf;
        P.sweight = m->sweight.p;
        P.ecdf = ecdf;
        P.rowpos = rowpos;
        P.key0 = (uint32_t)(m->cfg.seed & 0xffffffffu);
        P.key1 = key1;
        P.n_packets = (uint64_t)np;
        P.packet_base = 0;
        P.pool = misc + MISC_POOL;
        P.eps0 = eps0;
        P.max_events = m->cfg.max_events;
        // 0: the mode's default -- a per-lane walk handles events once 16 lanes
        // wait; a tile walk waits for every lane (its walks are short and alike)
        P.defer_lanes = m->cfg.defer_lanes > 0 ? m->cfg.defer_lanes : (m->cfg.transport_mode == 1 ? 64 : 16);
        P.acc = m->acc.p;
        P.acc_stride = m->acc_copies > 1 ? m->acc_stride : 0;
        P.acc2 = m->cfg.want_noise ? m->acc2.p : nullptr;
        P.binning = binning;
        P.n_incl = m->n_incl;
        P.sed_sum = m->sed_sum.p;
        P.sed_sum2 = m->sed_sum2.p;
        P.sed_n = m->sed_n.p;
        P.n_img = m->n_img;
        P.npix = m->npix;
        P.img_hw = m->img_hw;
        P.img_of_bin = m->img_of_bin.p;
        P.img_sum = m->img_sum.p;
        P.img_sum2 = m->img_sum2.p;
        P.n_peel = m->n_peel;
        P.peel_dir = m->peel_dir.p;
        P.rho_lin = f32 ? (const R*)(const void*)m->rho32.p : (const R*)(const void*)m->rho64.p;
        P.mrw_gamma = m->cfg.mrw_gamma;
        P.Tcell = m->T.p;
        P.mrw_tab = m->mrw_tab.p;
        P.mrw_ytab = m->mrw_ytab.p;
        P.psed_sum = m->psed_sum.p;
        P.psed_sum2 = m->psed_sum2.p;
        P.pimg_sum = m->pimg_sum.p;
        P.pimg_sum2 = m->pimg_sum2.p;
        P.ev_packets = m->ev_packets;
        P.ev_cap = m->ev_cap;
        P.evlog = m->evlog.p;
        P.evcount = m->evcount.p;
        P.counters = misc + MISC_CNT;
        P.energies = m->energies.p;
    }
}

int persistent_blocks(const mcrt_model* m, int bpc, int64_t np, int threads) {
    int64_t blocks = (int64_t)m->n_cu * bpc;
    const int64_t need = (np + threads - 1) / threads;
    if (blocks > need) blocks = need;
    return (int)(blocks < 1 ? 1 : blocks);
}

// Tiled sweeps (transport_mode 1).  Each step: the refill decision and the
// emission (device side), the scan of the per-tile counts, the grouping of
// the entries by tile, and one sweep, which writes the records still in
// flight into the other buffer.  The pool is refilled whenever fewer than
// `batch` records remain after a sweep, so only the end of the pass drains.
// The host never waits for a step: it copies each step's termination flag
// into pinned memory and checks the flag of the step kSweepLag-1 steps back,
// so that at most that many empty steps run after the last record.
constexpr int64_t kSweepBatch = 1ll << 25;  // default packets emitted at once
constexpr int64_t kSweepDrain = 1ll << 18;  // default records left for the per-lane finish
constexpr int64_t kMaxSweeps = 1ll << 20;    // every visit advances a packet; this is a backstop
constexpr int kSweepLag = 4;
constexpr int64_t kChunkSlots = 64;     // record slots of a chunk (as in the sweep kernels)

template <typename R>
mcrt_status run_sweeps(mcrt_model* m, TransportParams<R>& P, int64_t np, int64_t* n_sweeps,
                       int64_t* n_visits, double* ms_sweep, int64_t* n_drained) {
    hipStream_t s = m->stream;
    constexpr bool f32 = std::is_same<R, float>::value;
    for (int a = 0; a < 3; ++a)
        if (m->n[a] > 1024)
            return fail(m, MCRT_E_UNSUPPORTED,
                        "tiled sweeps hold at most 1024 cells per axis; use transport_mode 0");
    SweepParams S{};
    // tile shape and group size, 0 = by precision: FP32 24x24x20 tiles (FP32
    // density and FP64 tally, 135 KB of LDS) walked by one group of 512
    // threads per compute unit; FP64 16x16x32 tiles and 256 threads (its
    // register budget)
    S.txy = m->cfg.tile_xy == 0 ? (f32 ? 24 : 16) : m->cfg.tile_xy;
    S.tz = m->cfg.tile_z == 0 ? (f32 ? 20 : 32) : m->cfg.tile_z;
    const bool noise = P.acc2 != nullptr;
    // logging, binning, peeling and the modified random walk need the full
    // event code; a plain Lucy iteration runs the lean kernels
    const bool full = P.binning || P.mrw_gamma > 0.0 || P.ev_packets > 0;
    // LDS: tile density and tally (and sum of squares), the bins' chi, kappa,
    // albedo and g, and the staged tables; a tile too deep for LDS is halved in z
    const size_t tab_lds = (size_t)(m->src.size() + (kRows + m->src.size()) * m->ngroup) * sizeof(R);
    auto tile_bytes = [&](int tz) {
        return (size_t)S.txy * S.txy * tz * (sizeof(R) + (noise ? 2 : 1) * sizeof(double)) +
               4 * m->kap.size() * sizeof(R) + tab_lds;
    };
    while (tile_bytes(S.tz) > m->lds_max && S.tz > 1) S.tz /= 2;
    if (S.txy < 1 || S.txy > 64 || S.tz < 1 || S.tz > 64)
        return fail(m, MCRT_E_ARG, "tile extents must be in [1, 64] cells");
    S.mxy = (65536u + (unsigned)S.txy - 1u) / (unsigned)S.txy;
    S.mz = (65536u + (unsigned)S.tz - 1u) / (unsigned)S.tz;
    S.ntx = (m->n[0] + S.txy - 1) / S.txy;
    S.nty = (m->n[1] + S.txy - 1) / S.txy;
    S.ntz = (m->n[2] + S.tz - 1) / S.tz;
    S.ntiles = S.ntx * S.nty * S.ntz;
    S.visit_events = m->cfg.visit_events > 0 ? m->cfg.visit_events : 256;
    const size_t lds = tile_bytes(S.tz);
    if (lds > m->lds_max)
        return fail(m, MCRT_E_UNSUPPORTED, "tile and tables do not fit in LDS; use smaller tiles or fewer sources");
    // threads per group, 0 = by kernel: FP32 768 for the lean kernel (three
    // waves per SIMD hide the walk's LDS and the events' memory latency), 512
    // for the full one (its register budget); FP64 256
    int threads = m->cfg.block_size > 0 ? m->cfg.block_size : (f32 ? (full ? 512 : 768) : 256);
    if (full && threads > 512) threads = 512;
    // a work item: entries of one tile, about 16 records per thread when full
    S.item_ent = std::max(1, std::min(threads * 16 / 64, 256));
    // lanes of a wave that wait (events, escapes, exits, free lanes with a
    // record to take) before the wave handles them (40 on the 256^3 clump:
    // 0.6 % faster than 48, 2 % faster than 32)
    S.service = m->cfg.defer_lanes > 0 ? m->cfg.defer_lanes : 40;
    // packets emitted at a time: by default as many as two record buffers of
    // about 2.7 batches each hold within 30 % of the device's memory (FP32:
    // 2e8 packets on 288 GB), so that a pass of up to that many packets is
    // emitted at once; every tile then starts with its share of the whole
    // pass, the sweeps' visits serve the most records, and no refill tails
    // follow one another (on the 256^3 clump at 1e8 packets: 110 ms per
    // iteration, against 137 ms in batches of 2^25)
    int64_t batch = m->cfg.sweep_batch;
    if (batch <= 0) {
        const double per = 2.0 * 2.7 * (double)sweep_record_bytes(f32 ? 1 : 0);
        batch = std::max<int64_t>(kSweepBatch, (int64_t)(0.3 * (double)m->mem_total / per));
        batch = std::min<int64_t>(batch, (int64_t)1 << 30);
    }
    batch = std::min<int64_t>(batch, np);
    S.batch = (unsigned long long)batch;
    S.n_packets = (unsigned long long)np;
    // the tail: records left once every packet is emitted, finished per lane
    // (default: 2^18, at most 1/64 of the pass, so that small passes still
    // walk nearly all of their packets through the tiles)
    S.drain_below = m->cfg.sweep_drain < 0 ? 0ull
                    : m->cfg.sweep_drain == 0 ? (unsigned long long)std::min<int64_t>(kSweepDrain, np / 64)
                                              : (unsigned long long)m->cfg.sweep_drain;
    HIPCHK(sweep_prepare<R>(noise, full, lds));
    const int bpc = m->cfg.blocks_per_cu > 0 ? m->cfg.blocks_per_cu
                                             : sweep_max_blocks_per_cu<R>(noise, full, threads, lds);
    const int blocks = m->n_cu * bpc;
    // record slots per buffer: the records in flight (< 2 batch after a refill)
    // plus the slots left empty in chunks that a wave registers partly filled:
    // at most 7 chunks per wave and tile change, a group changes tile at most
    // once per work item, and a sweep has at most about (records / 32) /
    // item_ent work items (entries at least half full) plus one per tile.  A
    // pass that still runs out of slots stops with MCRT_E_NOMEM.
    // Each wave also holds up to one run of 1024 slots and 32 entry slots.
    const int64_t waves = (int64_t)blocks * (threads / 64);
    const int64_t items = 2 * batch / ((int64_t)S.item_ent * (kChunkSlots / 2)) + S.ntiles;
    const int64_t slack = kChunkSlots * 7 * (threads / 64) * (items + blocks);
    int64_t cap = 2 * batch + std::max<int64_t>(2 * batch / 3, slack) + 1024 * waves;
    cap = (cap + 63) / 64 * 64;
    if (cap > (int64_t)0xffff0000ll) return fail(m, MCRT_E_UNSUPPORTED, "sweep_batch too large for the record buffers");
    S.cap = (unsigned)cap;
    S.max_ent = (unsigned)std::min<int64_t>(cap / 4 + 65536 + 32 * waves, 0xffff0000ll);
    const size_t rq = sweep_record_bytes(f32 ? 1 : 0) / 16;
    for (int b = 0; b < 2; ++b) {
        HIPCHK(m->sw_rec[b].ensure(m->device, (size_t)cap * rq));
        HIPCHK(m->sw_ent_tile[b].ensure(m->device, S.max_ent));
        HIPCHK(m->sw_ent[b].ensure(m->device, S.max_ent));
        S.recs[b] = m->sw_rec[b].p;
        S.ent_tile[b] = m->sw_ent_tile[b].p;
        S.ent[b] = m->sw_ent[b].p;
    }
    HIPCHK(m->sw_sent.ensure(m->device, S.max_ent));
    HIPCHK(m->sw_tile_rec.ensure((size_t)S.ntiles));
    HIPCHK(m->sw_tile_ent.ensure((size_t)S.ntiles));
    HIPCHK(m->sw_ent_off.ensure((size_t)S.ntiles + 1));
    // work items: at most one per item_ent entries of a tile plus one per tile
    HIPCHK(m->sw_item_desc.ensure((size_t)S.max_ent / (size_t)S.item_ent + (size_t)S.ntiles + 1));
    HIPCHK(m->sw_cursor.ensure((size_t)S.ntiles));
    HIPCHK(m->sw_ctl.ensure(1));
    if (!m->sw_host) HIPCHK(hipHostMalloc((void**)&m->sw_host, kSweepLag * sizeof(unsigned), hipHostMallocDefault));
    for (int i = 0; i < kSweepLag; ++i)
        if (!m->sw_ev[i]) HIPCHK(hipEventCreateWithFlags(&m->sw_ev[i], hipEventDisableTiming));
    S.sent = m->sw_sent.p;
    S.tile_rec = m->sw_tile_rec.p;
    S.tile_ent = m->sw_tile_ent.p;
    S.ent_off = m->sw_ent_off.p;
    S.item_desc = m->sw_item_desc.p;
    S.cursor = m->sw_cursor.p;
    S.ctl = m->sw_ctl.p;
    HIPCHK(launch_fill_u32(S.tile_rec, S.ntiles, 0u, s));
    HIPCHK(launch_fill_u32(S.tile_ent, S.ntiles, 0u, s));
    HIPCHK(launch_fill_u32(reinterpret_cast<unsigned*>(S.ctl), (int)(sizeof(SweepCtl) / 4), 0u, s));
    const int64_t eb = (batch + sweep_emit_step() - 1) / sweep_emit_step();
    const int emit_blocks = (int)std::min<int64_t>(eb, (int64_t)m->n_cu * 4);
    const int group_blocks = m->n_cu * 4;
    P.packet_base = 0;
    int b = 0;  // the buffer the step's refill and sweep read
    bool done = false;
    int64_t step = 0;
    for (; !done; ++step) {
        if (step > kMaxSweeps) return fail(m, MCRT_E_DEVICE, "tiled sweeps did not finish");
        // the sweep kernel of every step is timed by a pair of events
        if ((size_t)(2 * step + 2) > m->sw_kev.size()) {
            for (int i = 0; i < 2; ++i) {
                hipEvent_t e;
                HIPCHK(hipEventCreate(&e));
                m->sw_kev.push_back(e);
            }
        }
        HIPCHK(launch_sweep_step<R>(P, S, b, full, emit_blocks, group_blocks, blocks, threads, lds, s,
                                    m->sw_kev[2 * step], m->sw_kev[2 * step + 1]));
        const int slot = (int)(step % kSweepLag);
        HIPCHK(hipMemcpyAsync(m->sw_host + slot, &S.ctl->done, sizeof(unsigned), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(m->sw_ev[slot], s));
        b ^= 1;
        if (step >= kSweepLag - 1) {
            const int k = (int)((step - (kSweepLag - 1)) % kSweepLag);
            HIPCHK(hipEventSynchronize(m->sw_ev[k]));
            done = m->sw_host[k] != 0u;
        }
    }
    SweepCtl c;
    HIPCHK(hipMemcpyAsync(&c, S.ctl, sizeof c, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double ms = 0.0;
    for (int64_t i = 0; i < step; ++i) {
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, m->sw_kev[2 * i], m->sw_kev[2 * i + 1]));
        ms += t;
    }
    if (c.drain) {
        // the per-lane finish of the tail, timed with the sweeps (its packets'
        // crossings count in the pass's algorithmic bytes)
        HIPCHK(hipEventRecord(m->sw_kev[0], s));
        HIPCHK(launch_sweep_drain<R>(P, S, (int)c.drain_buf, m->n_cu * 8, s));
        HIPCHK(hipEventRecord(m->sw_kev[1], s));
        HIPCHK(hipEventSynchronize(m->sw_kev[1]));
        float t = 0.f;
        HIPCHK(hipEventElapsedTime(&t, m->sw_kev[0], m->sw_kev[1]));
        ms += t;
    }
    *ms_sweep = ms;
    if (c.overflow & 2u) return fail(m, MCRT_E_DEVICE, "tiled sweeps: a record was not in its tile");
    if (c.overflow)
        return fail(m, MCRT_E_NOMEM, "tiled sweep record buffers overflowed; lower sweep_batch");
    *n_sweeps = (int64_t)c.sweeps;
    *n_visits = (int64_t)c.visits;
    *n_drained = c.drain ? (int64_t)c.drain_recs : 0;
    return MCRT_OK;
}

// Emission rows from T, zeroed tallies, then one persistent transport launch
// (or the tiled sweeps).
mcrt_status run_transport(mcrt_model* m, int64_t np, uint32_t key1, int binning,
                          mcrt_iter_stats* st) {
    hipStream_t s = m->stream;
    const bool f32 = m->cfg.precision == MCRT_FP32_TRANSPORT;
    unsigned long long* misc = m->misc.p;
    mcrt_status r = set_weights(m, np);
    if (r != MCRT_OK) return r;
    r = prepare_pass(m, np, false, m->cfg.transport_mode == 0);
    if (r != MCRT_OK) return r;
    const int threads = m->cfg.block_size > 0 ? m->cfg.block_size : 256;
    const int K = walk_batch_of(m);
    const int layout = m->t_layout;
    HIPCHK(hipEventRecord(m->ev[0], s));
    if (m->cfg.transport_mode == 1) {
        int64_t sweeps = 0, visits = 0, drained = 0;
        double ms_sweep = 0.0;
        if (f32) {
            TransportParams<float> P;
            make_params(m, np, key1, binning, P);
            r = run_sweeps<float>(m, P, np, &sweeps, &visits, &ms_sweep, &drained);
        } else {
            TransportParams<double> P;
            make_params(m, np, key1, binning, P);
            r = run_sweeps<double>(m, P, np, &sweeps, &visits, &ms_sweep, &drained);
        }
        if (r != MCRT_OK) return r;
        st->n_sweeps = sweeps;
        st->n_visits = visits;
        st->n_drained = drained;
        st->ms_dominant = ms_sweep;
    } else if (f32) {
        TransportParams<float> P;
        make_params(m, np, key1, binning, P);
        const size_t lds = transport_lds_bytes<float>(P);
        const int bpc = m->cfg.blocks_per_cu > 0
                            ? m->cfg.blocks_per_cu
                            : transport_max_blocks_per_cu<float>(K, layout, threads, lds);
        HIPCHK(launch_transport<float>(P, K, layout, persistent_blocks(m, bpc, np, threads), threads, s));
    } else {
        TransportParams<double> P;
        make_params(m, np, key1, binning, P);
        const size_t lds = transport_lds_bytes<double>(P);
        const int bpc = m->cfg.blocks_per_cu > 0
                            ? m->cfg.blocks_per_cu
                            : transport_max_blocks_per_cu<double>(K, layout, threads, lds);
        HIPCHK(launch_transport<double>(P, K, layout, persistent_blocks(m, bpc, np, threads), threads, s));
    }
    HIPCHK(hipEventRecord(m->ev[1], s));
    // counters
    unsigned long long h[MISC_N];
    double e[2];
    HIPCHK(hipMemcpyAsync(h, misc, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(e, m->energies.p, sizeof e, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, m->ev[0], m->ev[1]));
    st->ms_transport = ms;
    if (m->cfg.transport_mode != 1) st->ms_dominant = ms;  // one persistent launch
    st->n_row_clamped = (int64_t)h[MISC_SCRATCH];
    st->n_cross_dust = (int64_t)h[MISC_CNT + C_CROSS_DUST];
    st->n_cross_empty = (int64_t)h[MISC_CNT + C_CROSS_EMPTY];
    st->n_scatter = (int64_t)h[MISC_CNT + C_SCATTER];
    st->n_absorb = (int64_t)h[MISC_CNT + C_ABSORB];
    st->n_escape = (int64_t)h[MISC_CNT + C_ESCAPE];
    st->n_killed = (int64_t)h[MISC_CNT + C_KILLED];
    st->n_mrw = (int64_t)h[MISC_CNT + C_MRW];
    st->e_escaped = e[0];
    st->e_killed = e[1];
    st->precision = m->cfg.precision;
    return MCRT_OK;
}

mcrt_status select_rank(mcrt_model* m, const double* v, uint64_t rank, double* out) {
    hipStream_t s = m->stream;
    unsigned long long init[3] = {0ull, (unsigned long long)rank, 0ull};
    unsigned long long* sel = m->misc.p + MISC_SEL;
    HIPCHK(hipMemcpyAsync(sel, init, sizeof init, hipMemcpyHostToDevice, s));
    HIPCHK(launch_select(m->ncell, v, sel, m->hist.p, grid_blocks(m, m->ncell), s));
    unsigned long long res[3];
    HIPCHK(hipMemcpyAsync(res, sel, sizeof res, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    double d;
    memcpy(&d, &res[0], sizeof d);
    *out = d;
    return MCRT_OK;
}

uint64_t nearest_rank(double p, int64_t n) {
    int64_t r = (int64_t)ceil(p * (double)n);
    if (r < 1) r = 1;
    if (r > n) r = n;
    return (uint64_t)(r - 1);
}

void make_cell_params(mcrt_model* m, CellParams& P) {
    P = CellParams{};
    P.ncell = m->ncell;
    for (int a = 0; a < 3; ++a) P.n[a] = m->n[a];
    P.brick = m->t_layout == 1;
    P.bx = m->bx;
    P.bxy = m->bx * m->by;
    P.eps_over_vol = (m->ltot / (double)m->cfg.n_packets) / m->vol;
    P.rho = m->rho64.p;
    P.acc = m->acc.p;
    P.acc_copies = m->acc_copies;
    P.acc_stride = m->acc_stride;
    P.acc2 = m->cfg.want_noise ? m->acc2.p : nullptr;
    P.adot = m->adot.p;
    P.adot_prev = m->adot_prev.p;
    P.adot_sig = m->adot_sig.p;
    P.T = m->T.p;
    P.T_prev = m->T_prev.p;
    P.sig_rel = m->sig_rel.p;
    P.sig_rel_prev = m->sig_rel_prev.p;
    P.valid = m->valid.p;
    P.valid_prev = m->valid_prev.p;
    P.lnA = m->lnA.p;
    P.slope = m->slope.p;
    P.dy = m->dy;
    P.have_prev = m->have_prev;
    P.want_noise = m->cfg.want_noise;
    P.noise_thres = m->cfg.conv_noise_thres;
    P.Rbuf = m->Rbuf.p;
    P.rbuf = m->rbuf.p;
    P.stats = m->misc.p + MISC_STATS;
}

// Adot, T and the convergence statistics after a Lucy pass (Eqs. 2-6).
mcrt_status update_cells(mcrt_model* m, mcrt_iter_stats* st) {
    hipStream_t s = m->stream;
    unsigned long long* stats = m->misc.p + MISC_STATS;
    HIPCHK(hipMemsetAsync(stats, 0, 8 * sizeof(unsigned long long), s));
    CellParams P;
    make_cell_params(m, P);
    HIPCHK(hipEventRecord(m->ev[2], s));
    HIPCHK(launch_update(P, grid_blocks(m, m->ncell), s));
    unsigned long long h[8];
    HIPCHK(hipMemcpyAsync(h, stats, sizeof h, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    st->n_r = (int64_t)h[0];
    st->n_mask = (int64_t)h[1];
    st->n_unsampled = (int64_t)h[2];
    st->n_t_clamped = (int64_t)h[3];
    double rmax;
    memcpy(&rmax, &h[4], sizeof rmax);
    if (st->n_r > 0) {
        mcrt_status r = select_rank(m, m->Rbuf.p, nearest_rank(m->cfg.conv_p, st->n_r), &st->q);
        if (r != MCRT_OK) return r;
    } else {
        st->q = INFINITY;
    }
    st->delta = (isfinite(st->q) && isfinite(m->q_prev))
                    ? (st->q > m->q_prev ? st->q / m->q_prev : m->q_prev / st->q)
                    : INFINITY;
    st->converged_q = st->q < m->cfg.conv_q_thres && st->delta < m->cfg.conv_d_thres;
    m->q_prev = st->q;
    if (st->n_mask > 0) {
        st->max_dT = rmax;
        mcrt_status r = select_rank(m, m->rbuf.p, nearest_rank(0.999, st->n_mask), &st->p999_dT);
        if (r != MCRT_OK) return r;
    } else {
        st->max_dT = INFINITY;
        st->p999_dT = INFINITY;
    }
    st->converged_dT = st->n_mask > 0 && st->max_dT < m->cfg.conv_dT_thres;
    HIPCHK(hipEventRecord(m->ev[3], s));
    HIPCHK(hipEventSynchronize(m->ev[3]));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, m->ev[2], m->ev[3]));
    st->ms_update = ms;
    m->have_prev = 1;
    return MCRT_OK;
}

bool finite_all(const double* v, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return false;
    return true;
}

}  // namespace

extern "C" {

mcrt_status mcrt_run_cfg_default(mcrt_run_cfg* c) {
    if (!c) return MCRT_E_ARG;
    memset(c, 0, sizeof *c);
    c->n_packets = 100000;
    c->n_packets_final = 0;
    c->n_iter = 5;
    c->precision = MCRT_FP64;
    c->seed = 1;
    c->t_init = 10.0;
    c->max_events = 1000000;
    c->conv_p = 0.999;
    c->conv_q_thres = 2.0;
    c->conv_d_thres = 1.1;
    c->conv_dT_thres = 0.01;
    c->conv_noise_thres = 0.002;
    c->event_log_cap = 256;
    c->block_size = 0;
    c->defer_lanes = 0;
    c->walk_batch = 4;
    c->grid_layout = 0;
    c->tally_copies = kMaxTallyCopies;
    c->transport_mode = 1;
    c->tile_z = 0;
    c->visit_events = 256;
    c->tile_xy = 0;
    return MCRT_OK;
}

mcrt_status mcrt_create(mcrt_model** out, int hip_device) {
    if (!out) return MCRT_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MCRT_E_DEVICE;
    if (hip_device < 0 || hip_device >= ndev) return MCRT_E_ARG;
    mcrt_model* m = new (std::nothrow) mcrt_model();
    if (!m) return MCRT_E_NOMEM;
    m->device = hip_device;
    if (hipSetDevice(hip_device) != hipSuccess || hipStreamCreate(&m->stream) != hipSuccess) {
        delete m;
        return MCRT_E_DEVICE;
    }
    m->own_stream = true;
    hipDeviceGetAttribute(&m->n_cu, hipDeviceAttributeMultiprocessorCount, hip_device);
    {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess) m->mem_total = tot;
    }
    {
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) == hipSuccess &&
            lds > 0)
            m->lds_max = (size_t)lds;
        m->lds_max -= 5120;  // static LDS of the kernels that take dynamic LDS
    }
    for (int i = 0; i < 4; ++i) hipEventCreate(&m->ev[i]);
    // the device address of this device's staging array for the entry point
    // that allocates nothing (a failure is reported by that entry point)
    scratch_setup(hip_device);
    mcrt_run_cfg_default(&m->cfg);
    *out = m;
    return MCRT_OK;
}

void mcrt_destroy(mcrt_model* m) {
    if (!m) return;
    hipSetDevice(m->device);
    if (m->stream) hipStreamSynchronize(m->stream);
    for (int i = 0; i < 4; ++i)
        if (m->ev[i]) hipEventDestroy(m->ev[i]);
    m->rho64.release(); m->rho32.release(); m->rhoT64.release(); m->rhoT32.release();
    m->ecoarse64.release(); m->scoarse64.release(); m->ecoarse32.release(); m->scoarse32.release();
    m->chi64.release(); m->kap64.release(); m->alb64.release(); m->g64.release();
    m->lcdf64.release(); m->scdf64.release(); m->ecdf64.release();
    m->chi32.release(); m->kap32.release(); m->alb32.release(); m->g32.release();
    m->lcdf32.release(); m->scdf32.release(); m->ecdf32.release();
    m->spos.release(); m->scell.release(); m->sfrac.release(); m->sweight.release(); m->lnA.release(); m->slope.release();
    m->img_of_bin.release();
    m->acc.release(); m->acc2.release(); m->adot.release(); m->adot_prev.release();
    m->adot_sig.release(); m->T.release(); m->T_prev.release(); m->sig_rel.release();
    m->sig_rel_prev.release(); m->valid.release(); m->valid_prev.release();
    m->rowpos64.release(); m->rowpos32.release(); m->Rbuf.release(); m->rbuf.release();
    m->sed_sum.release(); m->sed_sum2.release(); m->sed_n.release();
    m->img_sum.release(); m->img_sum2.release(); m->evlog.release(); m->evcount.release();
    m->peel_dir.release(); m->psed_sum.release(); m->psed_sum2.release();
    m->pimg_sum.release(); m->pimg_sum2.release();
    m->ray_cube.release(); m->ray_sed.release(); m->ray_nu.release(); m->ray_lsrc.release();
    m->ray_btab.release();
    m->mrw_tab.release();
    m->mrw_ytab.release();
    m->pda_flag.release(); m->pda_vec.release(); m->pda_red.release(); m->pda_count.release();
    m->misc.release(); m->energies.release(); m->hist.release();
    for (int b = 0; b < 2; ++b) {
        m->sw_rec[b].release();
        m->sw_ent_tile[b].release();
        m->sw_ent[b].release();
    }
    m->sw_sent.release(); m->sw_tile_rec.release(); m->sw_tile_ent.release(); m->sw_ent_off.release();
    m->sw_item_desc.release(); m->sw_cursor.release(); m->sw_ctl.release();
    if (m->sw_host) hipHostFree(m->sw_host);
    for (int i = 0; i < 4; ++i)
        if (m->sw_ev[i]) hipEventDestroy(m->sw_ev[i]);
    for (hipEvent_t e : m->sw_kev) hipEventDestroy(e);
    if (m->own_stream && m->stream) hipStreamDestroy(m->stream);
    delete m;
}

const char* mcrt_last_error(const mcrt_model* m) { return m ? m->err.c_str() : "null model"; }

mcrt_status mcrt_set_stream(mcrt_model* m, void* hip_stream) {
    if (!m) return MCRT_E_ARG;
    hipSetDevice(m->device);
    hipStreamSynchronize(m->stream);
    if (m->own_stream && m->stream) hipStreamDestroy(m->stream);
    if (hip_stream) {
        m->stream = (hipStream_t)hip_stream;
        m->own_stream = false;
    } else {
        if (hipStreamCreate(&m->stream) != hipSuccess) return fail(m, MCRT_E_DEVICE, "stream");
        m->own_stream = true;
    }
    return MCRT_OK;
}

mcrt_status mcrt_set_grid(mcrt_model* m, int nx, int ny, int nz, const double lo[3],
                          const double hi[3]) {
    if (!m) return MCRT_E_ARG;
    if (nx < 1 || ny < 1 || nz < 1) return fail(m, MCRT_E_ARG, "grid dimensions must be >= 1");
    if ((int64_t)nx * ny * nz > (int64_t)INT32_MAX)
        return fail(m, MCRT_E_ARG, "grid has more than 2^31-1 cells");
    if (!lo || !hi) return fail(m, MCRT_E_ARG, "null bounds");
    for (int a = 0; a < 3; ++a)
        if (!(hi[a] > lo[a]) || !isfinite(lo[a]) || !isfinite(hi[a]))
            return fail(m, MCRT_E_ARG, "grid bounds must be finite with hi > lo");
    hipSetDevice(m->device);
    m->n[0] = nx; m->n[1] = ny; m->n[2] = nz;
    m->vol = 1.0;
    for (int a = 0; a < 3; ++a) {
        m->lo[a] = lo[a];
        m->hi[a] = hi[a];
        m->dx[a] = (hi[a] - lo[a]) / m->n[a];
        m->vol *= m->dx[a];
    }
    m->ncell = (int64_t)nx * ny * nz;
    m->have_grid = true;
    m->have_rho = false;
    m->state_ready = false;
    m->t_layout = -1;
    m->src.clear();
    m->tables_dirty = true;
    return MCRT_OK;
}

mcrt_status mcrt_set_density(mcrt_model* m, const double* rho, size_t n) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_grid) return fail(m, MCRT_E_STATE, "set the grid first");
    if (!rho) return fail(m, MCRT_E_ARG, "null density");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "density size does not match the grid");
    for (size_t i = 0; i < n; ++i)
        if (!(rho[i] >= 0.0) || !isfinite(rho[i]))
            return fail(m, MCRT_E_ARG, "density must be finite and >= 0");
    hipSetDevice(m->device);
    m->t_layout = -1;  // transport-layout copies are rebuilt from the new density
    HIPCHK(m->rho64.ensure(n));
    HIPCHK(m->rho32.ensure(n));
    HIPCHK(hipMemcpyAsync(m->rho64.p, rho, n * sizeof(double), hipMemcpyHostToDevice, m->stream));
    HIPCHK(launch_to_f32(m->ncell, m->rho64.p, m->rho32.p, grid_blocks(m, m->ncell), m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    m->have_rho = true;
    return MCRT_OK;
}

mcrt_status mcrt_set_density_device(mcrt_model* m, const void* d_rho, int is_fp64, size_t n) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_grid) return fail(m, MCRT_E_STATE, "set the grid first");
    if (!d_rho) return fail(m, MCRT_E_ARG, "null density");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "density size does not match the grid");
    hipSetDevice(m->device);
    m->t_layout = -1;  // transport-layout copies are rebuilt from the new density
    HIPCHK(m->rho64.ensure(n));
    HIPCHK(m->rho32.ensure(n));
    hipStream_t s = m->stream;
    const int b = grid_blocks(m, m->ncell);
    if (is_fp64) {
        HIPCHK(hipMemcpyAsync(m->rho64.p, d_rho, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
        HIPCHK(launch_to_f64(m->ncell, (const float*)d_rho, m->rho64.p, b, s));
    }
    HIPCHK(launch_to_f32(m->ncell, m->rho64.p, m->rho32.p, b, s));
    HIPCHK(m->misc.ensure(MISC_N));
    HIPCHK(hipMemsetAsync(m->misc.p + MISC_SCRATCH, 0, sizeof(unsigned long long), s));
    HIPCHK(launch_check_rho(m->ncell, m->rho64.p, m->misc.p + MISC_SCRATCH, b, s));
    unsigned long long bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, m->misc.p + MISC_SCRATCH, sizeof bad, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (bad) {
        m->have_rho = false;
        return fail(m, MCRT_E_ARG, "density must be finite and >= 0");
    }
    m->have_rho = true;
    return MCRT_OK;
}

mcrt_status mcrt_set_frequencies(mcrt_model* m, const double* nu_edges, int n_nu) {
    if (!m) return MCRT_E_ARG;
    if (n_nu < 1 || !nu_edges) return fail(m, MCRT_E_ARG, "need at least one frequency bin");
    for (int k = 0; k <= n_nu; ++k)
        if (!(nu_edges[k] > 0.0) || !isfinite(nu_edges[k]))
            return fail(m, MCRT_E_ARG, "frequency edges must be finite and > 0");
    for (int k = 0; k < n_nu; ++k)
        if (!(nu_edges[k + 1] > nu_edges[k])) return fail(m, MCRT_E_ARG, "frequency edges must increase");
    if (!m->src.empty()) return fail(m, MCRT_E_STATE, "set frequencies before adding sources");
    m->nu.assign(nu_edges, nu_edges + n_nu + 1);
    m->have_nu = true;
    m->have_dust = false;
    m->have_obs = false;
    m->tables_dirty = true;
    return MCRT_OK;
}

mcrt_status mcrt_set_dust(mcrt_model* m, const double* chi, const double* albedo, const double* g,
                          int n_nu) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_nu || n_nu != (int)m->nu.size() - 1)
        return fail(m, MCRT_E_SIZE, "dust size does not match the frequency bins");
    if (!chi || !albedo || !g) return fail(m, MCRT_E_ARG, "null dust array");
    bool any = false;
    for (int k = 0; k < n_nu; ++k) {
        if (!(chi[k] >= 0.0) || !isfinite(chi[k])) return fail(m, MCRT_E_ARG, "chi must be finite and >= 0");
        if (!(albedo[k] >= 0.0 && albedo[k] <= 1.0)) return fail(m, MCRT_E_ARG, "albedo must be in [0,1]");
        if (!(fabs(g[k]) < 1.0)) return fail(m, MCRT_E_ARG, "|g| must be < 1");
        any |= chi[k] * (1.0 - albedo[k]) > 0.0;
    }
    if (!any) return fail(m, MCRT_E_ARG, "dust must absorb in at least one bin");
    m->chi.assign(chi, chi + n_nu);
    m->alb.assign(albedo, albedo + n_nu);
    m->g.assign(g, g + n_nu);
    m->kap.resize(n_nu);
    for (int k = 0; k < n_nu; ++k) m->kap[k] = chi[k] * (1.0 - albedo[k]);
    m->have_dust = true;
    m->tables_dirty = true;
    return MCRT_OK;
}

static mcrt_status add_source(mcrt_model* m, const double pos[3], double lum,
                              const std::vector<double>& spec) {
    if (!m->have_grid || !m->have_nu)
        return fail(m, MCRT_E_STATE, "set grid and frequencies before sources");
    if (!pos) return fail(m, MCRT_E_ARG, "null position");
    if (!(lum > 0.0) || !isfinite(lum)) return fail(m, MCRT_E_ARG, "luminosity must be > 0");
    for (int a = 0; a < 3; ++a)
        if (!(pos[a] >= m->lo[a] && pos[a] < m->hi[a]))
            return fail(m, MCRT_E_ARG, "source outside the grid");
    double s = 0.0;
    for (double v : spec) {
        if (!(v >= 0.0) || !isfinite(v)) return fail(m, MCRT_E_ARG, "spectrum must be finite and >= 0");
        s += v;
    }
    if (!(s > 0.0)) return fail(m, MCRT_E_ARG, "spectrum has no power in the frequency bins");
    Source src;
    for (int a = 0; a < 3; ++a) src.pos[a] = pos[a];
    src.lum = lum;
    src.spec = spec;
    m->src.push_back(src);
    m->tables_dirty = true;
    return MCRT_OK;
}

mcrt_status mcrt_add_point_source(mcrt_model* m, const double pos[3], double lum, double teff) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_nu) return fail(m, MCRT_E_STATE, "set frequencies before sources");
    if (!(teff > 0.0) || !isfinite(teff)) return fail(m, MCRT_E_ARG, "temperature must be > 0");
    std::vector<double> spec;
    blackbody_bins(m->nu, teff, spec);
    return add_source(m, pos, lum, spec);
}

mcrt_status mcrt_add_point_source_spectrum(mcrt_model* m, const double pos[3], double lum,
                                           const double* l_nu_bin, int n_nu) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_nu || n_nu != (int)m->nu.size() - 1 || !l_nu_bin)
        return fail(m, MCRT_E_SIZE, "spectrum size does not match the bins");
    return add_source(m, pos, lum, std::vector<double>(l_nu_bin, l_nu_bin + n_nu));
}

mcrt_status mcrt_set_observers(mcrt_model* m, int n_incl, int img_npix, double img_half_width,
                               const int* img_nu_bins, int n_img_nu) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_nu) return fail(m, MCRT_E_STATE, "set frequencies before observers");
    if (n_incl < 1) return fail(m, MCRT_E_ARG, "need at least one inclination bin");
    if (n_img_nu < 0 || (n_img_nu > 0 && (img_npix < 1 || !(img_half_width > 0.0) || !img_nu_bins)))
        return fail(m, MCRT_E_ARG, "bad image parameters");
    const int nb = (int)m->nu.size() - 1;
    std::vector<int> seen(nb, 0);
    for (int i = 0; i < n_img_nu; ++i) {
        if (img_nu_bins[i] < 0 || img_nu_bins[i] >= nb) return fail(m, MCRT_E_ARG, "image bin out of range");
        if (seen[img_nu_bins[i]]++) return fail(m, MCRT_E_ARG, "duplicate image bin");
    }
    m->n_incl = n_incl;
    m->n_img = n_img_nu;
    m->npix = n_img_nu > 0 ? img_npix : 0;
    m->img_hw = img_half_width;
    m->img_bins.assign(img_nu_bins, img_nu_bins + n_img_nu);
    m->have_obs = true;
    m->tables_dirty = true;
    hipSetDevice(m->device);
    mcrt_status s = ensure_bins(m);
    if (s != MCRT_OK) return s;
    return clear_bins(m);
}

mcrt_status mcrt_set_peeloff(mcrt_model* m, const double* dirs, int n) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_obs) return fail(m, MCRT_E_STATE, "set observers before peeling-off directions");
    if (n < 0 || (n > 0 && !dirs)) return fail(m, MCRT_E_ARG, "bad peeling-off directions");
    for (int i = 0; i < n; ++i) {
        const double r = sqrt(dirs[3 * i] * dirs[3 * i] + dirs[3 * i + 1] * dirs[3 * i + 1] +
                              dirs[3 * i + 2] * dirs[3 * i + 2]);
        if (!(fabs(r - 1.0) < 1e-9)) return fail(m, MCRT_E_ARG, "peeling-off directions must be unit vectors");
    }
    hipSetDevice(m->device);
    m->n_peel = n;
    HIPCHK(m->peel_dir.ensure((size_t)(n > 0 ? 3 * n : 3)));
    if (n > 0) HIPCHK(hipMemcpy(m->peel_dir.p, dirs, (size_t)3 * n * sizeof(double), hipMemcpyHostToDevice));
    mcrt_status s = ensure_bins(m);
    if (s != MCRT_OK) return s;
    s = clear_bins(m);
    if (s != MCRT_OK) return s;
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_peeled_sed(mcrt_model* m, double* sum, double* sum2, size_t n) {
    if (!m || !sum) return MCRT_E_ARG;
    const size_t nps = (size_t)m->n_peel * 2 * m->kap.size();
    if (n != nps) return fail(m, MCRT_E_SIZE, "peeled SED size is n_peel*2*n_nu");
    hipSetDevice(m->device);
    if (nps) {
        HIPCHK(hipMemcpyAsync(sum, m->psed_sum.p, nps * sizeof(double), hipMemcpyDeviceToHost, m->stream));
        if (sum2)
            HIPCHK(hipMemcpyAsync(sum2, m->psed_sum2.p, nps * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    }
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_peeled_images(mcrt_model* m, double* sum, double* sum2, size_t n) {
    if (!m || !sum) return MCRT_E_ARG;
    const size_t npi = (size_t)m->n_img * m->n_peel * m->npix * m->npix;
    if (n != npi) return fail(m, MCRT_E_SIZE, "peeled image size is n_img*n_peel*npix^2");
    hipSetDevice(m->device);
    if (npi) {
        HIPCHK(hipMemcpyAsync(sum, m->pimg_sum.p, npi * sizeof(double), hipMemcpyDeviceToHost, m->stream));
        if (sum2)
            HIPCHK(hipMemcpyAsync(sum2, m->pimg_sum2.p, npi * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    }
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_raytrace(mcrt_model* m, int npix, double half_width) {
    if (!m) return MCRT_E_ARG;
    if (m->n_peel <= 0) return fail(m, MCRT_E_STATE, "no observers: call mcrt_set_peeloff first");
    if (npix < 1 || npix > 65536 || !(half_width > 0.0) || !isfinite(half_width))
        return fail(m, MCRT_E_ARG, "npix must be in [1, 65536] and half_width > 0");
    hipSetDevice(m->device);
    mcrt_status r = ready(m);
    if (r != MCRT_OK) return r;
    const size_t nnu = m->kap.size(), ns = m->src.size();
    const size_t ncube = (size_t)m->n_peel * npix * npix * nnu;
    if (ncube > ((size_t)1 << 34) || (size_t)m->n_peel * npix * npix > ((size_t)1 << 32))
        return fail(m, MCRT_E_ARG, "image cube above 2^34 values or 2^32 pixels");
    HIPCHK(m->ray_cube.ensure(ncube));
    HIPCHK(m->ray_sed.ensure((size_t)m->n_peel * 2 * nnu));
    HIPCHK(m->ray_nu.ensure(nnu + 1));
    HIPCHK(m->ray_lsrc.ensure(ns * nnu));
    if (!m->ray_btab_ok) {
        std::vector<double> tab;
        ray_planck_table(m->nu, tab);
        HIPCHK(m->ray_btab.ensure(tab.size()));
        HIPCHK(hipMemcpy(m->ray_btab.p, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
        m->ray_btab_ok = true;
    }
    std::vector<double> lsrc(ns * nnu);
    for (size_t i = 0; i < ns; ++i) {
        double tot = 0.0;
        for (size_t k = 0; k < nnu; ++k) tot += m->src[i].spec[k];
        for (size_t k = 0; k < nnu; ++k) lsrc[i * nnu + k] = m->src[i].lum * m->src[i].spec[k] / tot;
    }
    hipStream_t s = m->stream;
    HIPCHK(hipMemcpyAsync(m->ray_nu.p, m->nu.data(), (nnu + 1) * sizeof(double), hipMemcpyHostToDevice, s));
    if (ns) HIPCHK(hipMemcpyAsync(m->ray_lsrc.p, lsrc.data(), ns * nnu * sizeof(double), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemsetAsync(m->ray_sed.p, 0, (size_t)m->n_peel * 2 * nnu * sizeof(double), s));
    RayParams R{};
    for (int a = 0; a < 3; ++a) {
        R.n[a] = m->n[a];
        R.lo[a] = m->lo[a];
        R.hi[a] = m->hi[a];
        R.dx[a] = m->dx[a];
    }
    R.rho = m->rho64.p;
    R.T = m->T.p;
    R.nnu = (int)nnu;
    R.nu = m->ray_nu.p;
    R.chi = m->chi64.p;
    R.kap = m->kap64.p;
    R.n_obs = m->n_peel;
    R.dirs = m->peel_dir.p;
    R.npix = npix;
    R.hw = half_width;
    R.nsrc = (int)ns;
    R.spos = m->spos.p;
    R.lsrc = m->ray_lsrc.p;
    R.cube = m->ray_cube.p;
    R.sed = m->ray_sed.p;
    R.btab = reinterpret_cast<const double2*>(m->ray_btab.p);
    R.dlnT = (log(kTHi) - log(kTLo)) / (kRayTRows - 1);
    HIPCHK(launch_raytrace(R, s));
    HIPCHK(hipStreamSynchronize(s));
    m->ray_npix = npix;
    return MCRT_OK;
}

mcrt_status mcrt_apply_pda(mcrt_model* m, double noise, int passes, mcrt_pda_stats* st) {
    if (!m || !st) return MCRT_E_ARG;
    if (!(noise > 0.0) || !isfinite(noise) || passes < 1 || passes > 100)
        return fail(m, MCRT_E_ARG, "noise must be > 0 and passes in [1, 100]");
    if (m->iter < 1) return fail(m, MCRT_E_STATE, "run a Lucy iteration first");
    hipSetDevice(m->device);
    mcrt_status r = ready(m);
    if (r != MCRT_OK) return r;
    memset(st, 0, sizeof *st);
    hipStream_t s = m->stream;
    if (!m->mrw_tab_built) {
        std::vector<double> tab;
        mean_opacity_table(m->nu, m->kap, m->chi, tab);
        HIPCHK(upload(m->mrw_tab, tab, s));
        HIPCHK(upload(m->mrw_ytab, escape_table(), s));
        HIPCHK(hipStreamSynchronize(s));
        m->mrw_tab_built = true;
    }
    const size_t nc = (size_t)m->ncell;
    HIPCHK(m->pda_flag.ensure(nc));
    HIPCHK(m->pda_vec.ensure(8 * nc));
    HIPCHK(m->pda_red.ensure(5));
    HIPCHK(m->pda_count.ensure(1));
    PdaParams P{};
    P.ncell = m->ncell;
    for (int a = 0; a < 3; ++a) {
        P.n[a] = m->n[a];
        P.dx[a] = m->dx[a];
    }
    P.rho = m->rho64.p;
    P.T = m->T.p;
    P.adot = m->adot.p;
    P.adot_sig = m->cfg.want_noise ? m->adot_sig.p : nullptr;
    P.noise = noise;
    P.mrw_tab = m->mrw_tab.p;
    P.lnA = m->lnA.p;
    P.slope = m->slope.p;
    P.dy = m->dy;
    P.flag = m->pda_flag.p;
    double* v = m->pda_vec.p;
    P.a = v;
    P.x = v + nc;
    P.r = v + 2 * nc;
    P.z = v + 3 * nc;
    P.p = v + 4 * nc;
    P.q = v + 5 * nc;
    P.diag = v + 6 * nc;
    P.b = v + 7 * nc;
    P.red = m->pda_red.p;
    P.count = m->pda_count.p;
    P.adot_out = m->adot.p;
    P.valid = m->valid.p;
    auto read_count = [&](unsigned* out) -> hipError_t {
        hipError_t e = hipMemcpyAsync(out, P.count, sizeof *out, hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return e;
        return hipStreamSynchronize(s);
    };
    for (int pass = 0; pass < passes; ++pass) {
        // the cells are chosen once, from the Monte-Carlo estimate; chi_R is
        // evaluated at the current temperatures on every pass
        HIPCHK(launch_fill_u32(P.count, 1, 0u, s));
        HIPCHK(launch_pda_coefficients(P, pass == 0 ? 1 : 0, s));
        if (pass == 0) {
            unsigned n_pda = 0;
            HIPCHK(read_count(&n_pda));
            st->n_pda = n_pda;
            if (n_pda == 0) break;
            for (unsigned round = 0; round <= n_pda; ++round) {
                HIPCHK(launch_fill_u32(P.count, 1, 0u, s));
                HIPCHK(launch_pda_connect(P, s));
                unsigned changed = 0;
                HIPCHK(read_count(&changed));
                st->n_solved += changed;
                if (changed == 0) break;
            }
            if (st->n_solved == 0) break;
        }
        HIPCHK(hipMemsetAsync(P.red, 0, 5 * sizeof(double), s));
        HIPCHK(launch_pda_init(P, s));
        double red[5];
        HIPCHK(hipMemcpyAsync(red, P.red, sizeof red, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const double bb = red[4];
        double rr = red[0] > 0.0 ? 1.0 : 0.0;  // nothing to do when the start solves it
        int it = 0;
        const int max_it = (int)std::min<int64_t>(100000, 10 * st->n_solved + 100);
        while (rr > 0.0 && it < max_it) {
            HIPCHK(launch_pda_iteration(P, s));
            HIPCHK(hipMemcpyAsync(&rr, P.red + 3, sizeof rr, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            ++it;
            if (!(rr > 1e-24 * bb)) break;  // relative residual 1e-12
            HIPCHK(launch_pda_shift(P, s));
        }
        st->cg_iterations = it;
        st->residual = bb > 0.0 ? sqrt(fmax(rr, 0.0) / bb) : 0.0;
        st->passes = pass + 1;
        HIPCHK(launch_pda_finish(P, s));
    }
    HIPCHK(hipStreamSynchronize(s));
    return MCRT_OK;
}

mcrt_status mcrt_get_raytraced_sed(mcrt_model* m, double* sed, size_t n) {
    if (!m || !sed) return MCRT_E_ARG;
    if (m->ray_npix == 0) return fail(m, MCRT_E_STATE, "no raytracing done");
    if (n != (size_t)m->n_peel * 2 * m->kap.size()) return fail(m, MCRT_E_SIZE, "raytraced SED size is n_peel*2*n_nu");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(sed, m->ray_sed.p, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_raytraced_cube(mcrt_model* m, double* cube, size_t n) {
    if (!m || !cube) return MCRT_E_ARG;
    if (m->ray_npix == 0) return fail(m, MCRT_E_STATE, "no raytracing done");
    if (n != (size_t)m->n_peel * m->ray_npix * m->ray_npix * m->kap.size())
        return fail(m, MCRT_E_SIZE, "raytraced cube size is n_peel*npix^2*n_nu");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(cube, m->ray_cube.p, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_raytraced_cube_device(mcrt_model* m, const double** d_cube) {
    if (!m || !d_cube) return MCRT_E_ARG;
    if (m->ray_npix == 0) return fail(m, MCRT_E_STATE, "no raytracing done");
    *d_cube = m->ray_cube.p;
    return MCRT_OK;
}

mcrt_status mcrt_set_run(mcrt_model* m, const mcrt_run_cfg* c) {
    if (!m || !c) return MCRT_E_ARG;
    if (c->n_packets < 1 || c->n_packets_final < 0) return fail(m, MCRT_E_ARG, "packet counts must be >= 1");
    if (c->n_iter < 0) return fail(m, MCRT_E_ARG, "n_iter must be >= 0");
    if (c->precision != MCRT_FP64 && c->precision != MCRT_FP32_TRANSPORT)
        return fail(m, MCRT_E_ARG, "unknown precision");
    if (!(c->t_init > 0.0) || !isfinite(c->t_init)) return fail(m, MCRT_E_ARG, "t_init must be > 0");
    if (c->max_events < 0) return fail(m, MCRT_E_ARG, "max_events must be >= 0");
    if (!(c->conv_p > 0.0 && c->conv_p <= 1.0)) return fail(m, MCRT_E_ARG, "conv_p must be in (0,1]");
    if (c->event_log_packets < 0 || c->event_log_cap < 0) return fail(m, MCRT_E_ARG, "bad event log size");
    if (c->block_size < 0 || c->block_size % 64 != 0 || c->block_size > 1024)
        return fail(m, MCRT_E_ARG, "block_size must be a multiple of 64");
    if (c->block_size > (c->transport_mode == 1 && c->precision == MCRT_FP32_TRANSPORT ? 768 : 256))
        return fail(m, MCRT_E_ARG, "block_size above 256 (768 for FP32 tiled sweeps) is not supported");
    if (c->defer_lanes < 0 || c->defer_lanes > 64) return fail(m, MCRT_E_ARG, "defer_lanes must be in [0,64]");
    if (c->blocks_per_cu < 0) return fail(m, MCRT_E_ARG, "blocks_per_cu must be >= 0");
    if (c->transport_mode != 0 && c->transport_mode != 1)
        return fail(m, MCRT_E_ARG, "transport_mode must be 0 or 1");
    if (c->tile_z < 0 || c->tile_z > 64) return fail(m, MCRT_E_ARG, "tile_z must be in [1, 64] (0: default)");
    if (c->visit_events < 0) return fail(m, MCRT_E_ARG, "visit_events must be >= 0");
    if (c->tile_xy != 0 && (c->tile_xy < 4 || c->tile_xy > 64 || c->tile_xy % 4 != 0))
        return fail(m, MCRT_E_ARG, "tile_xy must be a multiple of 4 in [4, 64] (0: default)");
    if (!(c->mrw_gamma >= 0.0) || !isfinite(c->mrw_gamma)) return fail(m, MCRT_E_ARG, "mrw_gamma must be >= 0");
    if (c->sweep_batch < 0 || c->sweep_batch > ((int64_t)1 << 30))
        return fail(m, MCRT_E_ARG, "sweep_batch must be in [0, 2^30]");
    if (c->sweep_drain < -1 || c->sweep_drain > ((int64_t)1 << 30))
        return fail(m, MCRT_E_ARG, "sweep_drain must be -1 or in [0, 2^30]");
    const bool reset = !m->have_run || c->t_init != m->cfg.t_init;
    m->cfg = *c;
    if (m->cfg.mrw_gamma > 0.0 && !m->mrw_tab_built) m->tables_dirty = true;
    if (m->cfg.event_log_cap == 0) m->cfg.event_log_cap = 256;
    if (m->cfg.conv_noise_thres <= 0.0) m->cfg.conv_noise_thres = 0.002;
    if (m->cfg.visit_events == 0) m->cfg.visit_events = 256;
    m->have_run = true;
    if (reset) m->state_ready = false;
    return MCRT_OK;
}

mcrt_status mcrt_set_temperature(mcrt_model* m, const double* T, size_t n) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_grid || !m->have_run) return fail(m, MCRT_E_STATE, "set grid and run parameters first");
    if (!T) return fail(m, MCRT_E_ARG, "null temperature");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "temperature size does not match the grid");
    for (size_t j = 0; j < n; ++j)
        if (!(T[j] > 0.0) || !isfinite(T[j])) return fail(m, MCRT_E_ARG, "temperature must be > 0");
    hipSetDevice(m->device);
    mcrt_status s = ensure_state(m);
    if (s != MCRT_OK) return s;
    HIPCHK(hipMemcpyAsync(m->T.p, T, n * sizeof(double), hipMemcpyHostToDevice, m->stream));
    const int b = grid_blocks(m, m->ncell);
    HIPCHK(launch_fill_u8(m->ncell, m->valid.p, 1, b, m->stream));
    HIPCHK(launch_fill_f64(m->ncell, m->sig_rel.p, 0.0, b, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    m->have_prev = 0;
    m->q_prev = INFINITY;
    return MCRT_OK;
}

mcrt_status mcrt_set_temperature_device(mcrt_model* m, const void* d_T, int is_fp64, size_t n) {
    if (!m) return MCRT_E_ARG;
    if (!m->have_grid || !m->have_run) return fail(m, MCRT_E_STATE, "set grid and run parameters first");
    if (!d_T) return fail(m, MCRT_E_ARG, "null temperature");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "temperature size does not match the grid");
    hipSetDevice(m->device);
    mcrt_status s = ensure_state(m);
    if (s != MCRT_OK) return s;
    hipStream_t st = m->stream;
    const int b = grid_blocks(m, m->ncell);
    if (is_fp64) HIPCHK(hipMemcpyAsync(m->T.p, d_T, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    else HIPCHK(launch_to_f64(m->ncell, (const float*)d_T, m->T.p, b, st));
    HIPCHK(hipMemsetAsync(m->misc.p + MISC_SCRATCH, 0, sizeof(unsigned long long), st));
    HIPCHK(launch_check_T(m->ncell, m->T.p, m->misc.p + MISC_SCRATCH, b, st));
    unsigned long long bad = 0;
    HIPCHK(hipMemcpyAsync(&bad, m->misc.p + MISC_SCRATCH, sizeof bad, hipMemcpyDeviceToHost, st));
    HIPCHK(launch_fill_u8(m->ncell, m->valid.p, 1, b, st));
    HIPCHK(launch_fill_f64(m->ncell, m->sig_rel.p, 0.0, b, st));
    HIPCHK(hipStreamSynchronize(st));
    if (bad) {
        m->state_ready = false;  // the next call starts again from t_init
        return fail(m, MCRT_E_ARG, "temperature must be finite and > 0");
    }
    m->have_prev = 0;
    m->q_prev = INFINITY;
    return MCRT_OK;
}

mcrt_status mcrt_iterate(mcrt_model* m, mcrt_iter_stats* st) {
    if (!m || !st) return MCRT_E_ARG;
    const double t0 = now_ms();
    hipSetDevice(m->device);
    mcrt_status s = ready(m);
    if (s != MCRT_OK) return s;
    memset(st, 0, sizeof *st);
    if (m->cfg.bin_every_iteration) {
        s = clear_bins(m);
        if (s != MCRT_OK) return s;
    }
    s = run_transport(m, m->cfg.n_packets, (uint32_t)m->iter, m->cfg.bin_every_iteration, st);
    if (s != MCRT_OK) return s;
    s = update_cells(m, st);
    if (s != MCRT_OK) return s;
    st->iteration = m->iter;
    m->iter++;
    st->ms_total = now_ms() - t0;
    return MCRT_OK;
}

mcrt_status mcrt_final_pass(mcrt_model* m, mcrt_iter_stats* st) {
    if (!m || !st) return MCRT_E_ARG;
    const double t0 = now_ms();
    hipSetDevice(m->device);
    mcrt_status s = ready(m);
    if (s != MCRT_OK) return s;
    memset(st, 0, sizeof *st);
    s = clear_bins(m);
    if (s != MCRT_OK) return s;
    const int64_t np = m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets;
    s = run_transport(m, np, 0x80000000u | (uint32_t)m->iter, 1, st);
    if (s != MCRT_OK) return s;
    st->iteration = m->iter;
    st->ms_total = now_ms() - t0;
    return MCRT_OK;
}

mcrt_status mcrt_run(mcrt_model* m, mcrt_run_stats* rs) {
    if (!m || !rs) return MCRT_E_ARG;
    memset(rs, 0, sizeof *rs);
    rs->first_converged = -1;
    const double t0 = now_ms();
    for (int i = 0; i < m->cfg.n_iter; ++i) {
        mcrt_status s = mcrt_iterate(m, &rs->last);
        if (s != MCRT_OK) return s;
        rs->n_iterations++;
        const bool conv = m->cfg.stop_on_convergence == 1   ? rs->last.converged_dT != 0
                          : m->cfg.stop_on_convergence == 2 ? rs->last.converged_q != 0
                                                            : false;
        if (conv && rs->first_converged < 0) {
            rs->first_converged = rs->last.iteration;
            rs->ms_to_converged = now_ms() - t0;
            rs->converged = 1;
            break;
        }
    }
    mcrt_status s = mcrt_final_pass(m, &rs->final_pass);
    if (s != MCRT_OK) return s;
    rs->ms_total = now_ms() - t0;
    return MCRT_OK;
}

mcrt_status mcrt_get_specific_energy(mcrt_model* m, double* adot, double* adot_sigma, size_t n) {
    if (!m || !adot) return MCRT_E_ARG;
    if (!m->state_ready) return fail(m, MCRT_E_STATE, "no iteration has run");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "buffer size does not match the grid");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(adot, m->adot.p, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    if (adot_sigma)
        HIPCHK(hipMemcpyAsync(adot_sigma, m->adot_sig.p, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_temperature(mcrt_model* m, double* T, size_t n) {
    if (!m || !T) return MCRT_E_ARG;
    if (!m->state_ready) return fail(m, MCRT_E_STATE, "no state yet");
    if ((int64_t)n != m->ncell) return fail(m, MCRT_E_SIZE, "buffer size does not match the grid");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(T, m->T.p, n * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_temperature_device(mcrt_model* m, const double** d_T) {
    if (!m || !d_T) return MCRT_E_ARG;
    if (!m->state_ready) return fail(m, MCRT_E_STATE, "no state yet");
    *d_T = m->T.p;
    return MCRT_OK;
}

mcrt_status mcrt_get_sed(mcrt_model* m, double* sum, double* sum2, int64_t* count, size_t n) {
    if (!m || !sum) return MCRT_E_ARG;
    const size_t ns = (size_t)m->n_incl * m->kap.size();
    if (!m->sed_sum.p) return fail(m, MCRT_E_STATE, "no SED yet");
    if (n != ns) return fail(m, MCRT_E_SIZE, "buffer size does not match n_incl*n_nu");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(sum, m->sed_sum.p, ns * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    if (sum2) HIPCHK(hipMemcpyAsync(sum2, m->sed_sum2.p, ns * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    if (count) HIPCHK(hipMemcpyAsync(count, m->sed_n.p, ns * sizeof(int64_t), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_images(mcrt_model* m, double* sum, double* sum2, size_t n) {
    if (!m) return MCRT_E_ARG;
    const size_t ni = (size_t)m->n_img * m->n_incl * m->npix * m->npix;
    if (n != ni) return fail(m, MCRT_E_SIZE, "buffer size does not match the images");
    if (ni == 0) return MCRT_OK;
    if (!sum) return MCRT_E_ARG;
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(sum, m->img_sum.p, ni * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    if (sum2) HIPCHK(hipMemcpyAsync(sum2, m->img_sum2.p, ni * sizeof(double), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_get_event_log(mcrt_model* m, mcrt_event* ev, size_t cap_total, int32_t* counts,
                               size_t n_counts) {
    if (!m || !ev || !counts) return MCRT_E_ARG;
    if (m->ev_packets <= 0) return fail(m, MCRT_E_STATE, "no event log");
    const size_t need = (size_t)m->ev_packets * m->ev_cap;
    if (cap_total != need || n_counts != (size_t)m->ev_packets)
        return fail(m, MCRT_E_SIZE, "event log buffers do not match packets*cap");
    hipSetDevice(m->device);
    HIPCHK(hipMemcpyAsync(ev, m->evlog.p, need * sizeof(mcrt_event), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipMemcpyAsync(counts, m->evcount.p, n_counts * sizeof(int32_t), hipMemcpyDeviceToHost, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    return MCRT_OK;
}

mcrt_status mcrt_scatter_directions(mcrt_model* m, int precision, const double* d, const double* mu,
                                    const double* phi, double* out, int n) {
    if (!m) return MCRT_E_ARG;
    if (precision != MCRT_FP64 && precision != MCRT_FP32_TRANSPORT)
        return fail(m, MCRT_E_ARG, "unknown precision");
    if (n < 0 || (n > 0 && (!d || !mu || !phi || !out))) return fail(m, MCRT_E_ARG, "bad direction arrays");
    if (n == 0) return MCRT_OK;
    for (int i = 0; i < n; ++i)
        if (!(mu[i] >= -1.0 && mu[i] <= 1.0) || !isfinite(phi[i]) || !isfinite(d[3 * i]) ||
            !isfinite(d[3 * i + 1]) || !isfinite(d[3 * i + 2]))
            return fail(m, MCRT_E_ARG, "mu must lie in [-1,1]; directions and phi finite");
    hipStream_t s = m->stream;
    struct Guard {
        DBuf<double> b;
        ~Guard() { b.release(); }
    } g;
    DBuf<double>& buf = g.b;
    HIPCHK(buf.ensure((size_t)9 * n));
    double* dd = buf.p;
    double* dm = dd + 3 * (size_t)n;
    double* dp = dm + n;
    double* dout = dp + n;
    HIPCHK(hipMemcpyAsync(dd, d, 3 * sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dm, mu, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dp, phi, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(launch_rotate(precision == MCRT_FP32_TRANSPORT ? 1 : 0, dd, dm, dp, dout, n, s));
    HIPCHK(hipMemcpyAsync(out, dout, 3 * sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MCRT_OK;
}

mcrt_status mcrt_scatter_directions_noalloc(mcrt_model* m, int precision, const double* d, const double* mu,
                                            const double* phi, double* out, int n) {
    if (!m) return MCRT_E_ARG;
    if (precision != MCRT_FP64 && precision != MCRT_FP32_TRANSPORT)
        return fail(m, MCRT_E_ARG, "unknown precision");
    if (n < 0 || (n > 0 && (!d || !mu || !phi || !out))) return fail(m, MCRT_E_ARG, "bad direction arrays");
    if (n > kNoAllocDirs)
        return fail(m, MCRT_E_SIZE, "at most 65536 directions per call (the static staging array)");
    if (n == 0) return MCRT_OK;
    for (int i = 0; i < n; ++i)
        if (!(mu[i] >= -1.0 && mu[i] <= 1.0) || !isfinite(phi[i]) || !isfinite(d[3 * i]) ||
            !isfinite(d[3 * i + 1]) || !isfinite(d[3 * i + 2]))
            return fail(m, MCRT_E_ARG, "mu must lie in [-1,1]; directions and phi finite");
    HIPCHK(hipSetDevice(m->device));
    double* base = scratch_ptr(m->device);
    if (!base) {
        HIPCHK(scratch_setup(m->device));
        base = scratch_ptr(m->device);
    }
    hipStream_t s = m->stream;
    // every element read below is written first in this call
    double* dd = base;
    double* dm = dd + 3 * (size_t)n;
    double* dp = dm + n;
    double* dout = dp + n;
    HIPCHK(hipMemcpyAsync(dd, d, 3 * sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dm, mu, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(dp, phi, sizeof(double) * n, hipMemcpyHostToDevice, s));
    HIPCHK(launch_rotate(precision == MCRT_FP32_TRANSPORT ? 1 : 0, dd, dm, dp, dout, n, s));
    HIPCHK(hipMemcpyAsync(out, dout, 3 * sizeof(double) * n, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return MCRT_OK;
}

mcrt_status mcrt_device_info(mcrt_model* m, int* n_cu, int* wave_size) {
    if (!m) return MCRT_E_ARG;
    if (n_cu) *n_cu = m->n_cu;
    if (wave_size) {
        int w = 64;
        hipDeviceGetAttribute(&w, hipDeviceAttributeWarpSize, m->device);
        *wave_size = w;
    }
    return MCRT_OK;
}

}  // extern "C"

// ===========================================================================
// Batching: the packets of many models in one persistent launch, iterations
// after the first replayed from a captured hipGraph, launch shape chosen by
// timing calibration runs (cached per workload class).
// ===========================================================================
namespace mcrt {
template <typename R>
hipError_t launch_transport_batch(const TransportParams<R>* Ps, const unsigned long long* chunk_start,
                                  int n_models, unsigned long long* pool, const uint32_t* keys,
                                  int K, int brick, int blocks, int threads, hipStream_t st);
template <typename R> int batch_max_blocks_per_cu(int K, int brick, int threads);
hipError_t launch_add_u32(int64_t n, uint32_t* p, uint32_t v, int blocks, hipStream_t st);
hipError_t launch_fill_u32(int64_t n, uint32_t* p, uint32_t v, int blocks, hipStream_t st);
}  // namespace mcrt

namespace {

struct LaunchShape {
    int block_size, walk_batch, defer, bpc;
};

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, LaunchShape> g_tune_cache;  // workload class -> shape

struct Batch {
    std::vector<mcrt_model*> ms;
    std::vector<hipStream_t> saved_streams;
    hipStream_t s = nullptr;
    bool f32 = false;
    int layout = 0;
    void* d_params = nullptr;
    unsigned long long* d_chunks = nullptr;  // n+1 prefix of 64-packet chunks, then the pool
    uint32_t* d_keys = nullptr;
    int n_cu = 256;
    ~Batch() {
        if (d_params) hipFree(d_params);
        if (d_chunks) hipFree(d_chunks);
        if (d_keys) hipFree(d_keys);
        for (size_t i = 0; i < ms.size() && i < saved_streams.size(); ++i) ms[i]->stream = saved_streams[i];
    }
    int n() const { return (int)ms.size(); }
    unsigned long long* pool() const { return d_chunks + ms.size() + 1; }
};

#define BCHK(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(B.ms[0], e_ == hipErrorOutOfMemory ? MCRT_E_NOMEM : MCRT_E_DEVICE,   \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                  \
    } while (0)

// Launch parameters of every model for a pass of frac * n_packets packets per
// model (frac = 1 for real passes), the chunk prefix and the per-model keys.
template <typename R>
mcrt_status batch_upload(Batch& B, double frac, int binning, const LaunchShape& sh,
                         const std::vector<uint32_t>& keys) {
    std::vector<TransportParams<R>> P(B.n());
    std::vector<unsigned long long> chunks(B.n() + 2, 0ull);
    for (int i = 0; i < B.n(); ++i) {
        mcrt_model* m = B.ms[i];
        int64_t np = binning ? (m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets)
                             : m->cfg.n_packets;
        if (frac < 1.0) np = std::max<int64_t>(64, (int64_t)(frac * (double)np));
        // the parameters point at buffers that set_weights and prepare_pass
        // allocate (source weights, emission rows, event log) and depend on the
        // tally copies prepare_pass selects
        mcrt_status r = set_weights(m, np);
        if (r != MCRT_OK) return r;
        r = prepare_pass(m, np, false, true);
        if (r != MCRT_OK) return r;
        make_params(m, np, 0u, binning, P[i]);
        P[i].lds_tables = 0;
        P[i].defer_lanes = sh.defer;
        chunks[i + 1] = chunks[i] + (unsigned long long)((np + kPoolChunk - 1) / kPoolChunk);
    }
    BCHK(hipMemcpy(B.d_params, P.data(), P.size() * sizeof(TransportParams<R>), hipMemcpyHostToDevice));
    BCHK(hipMemcpy(B.d_chunks, chunks.data(), chunks.size() * sizeof(unsigned long long),
                   hipMemcpyHostToDevice));
    BCHK(hipMemcpy(B.d_keys, keys.data(), keys.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    return MCRT_OK;
}

// Device work of one batched pass on B.s (capturable when graph_safe).
template <typename R>
mcrt_status batch_pass_ops(Batch& B, double frac, const LaunchShape& sh, bool graph_safe,
                           bool update, bool bump_keys) {
    for (int i = 0; i < B.n(); ++i) {
        mcrt_model* m = B.ms[i];
        int64_t np = m->cfg.n_packets;  // the same count batch_upload gave the model
        if (frac < 1.0) np = std::max<int64_t>(64, (int64_t)(frac * (double)np));
        mcrt_status r = prepare_pass(m, np, graph_safe, true);
        if (r != MCRT_OK) return r;
    }
    BCHK(launch_fill_u64(1, B.pool(), 0ull, 1, B.s));
    int64_t total_np = 0;
    for (mcrt_model* m : B.ms) total_np += m->cfg.n_packets;
    int64_t blocks = (int64_t)B.n_cu * sh.bpc;
    const int64_t need = ((int64_t)(frac * (double)total_np) + sh.block_size - 1) / sh.block_size;
    if (blocks > need) blocks = need;
    if (blocks < 1) blocks = 1;
    BCHK(launch_transport_batch<R>((const TransportParams<R>*)B.d_params, B.d_chunks, B.n(), B.pool(),
                                   B.d_keys, sh.walk_batch, B.layout, (int)blocks, sh.block_size,
                                   B.s));
    if (update) {
        for (mcrt_model* m : B.ms) {
            CellParams P;
            make_cell_params(m, P);
            BCHK(launch_fill_u64(8, m->misc.p + MISC_STATS, 0ull, 1, B.s));
            BCHK(launch_update(P, grid_blocks(m, m->ncell), B.s));
        }
    }
    if (bump_keys) BCHK(launch_add_u32(B.n(), B.d_keys, 1u, 1, B.s));
    return MCRT_OK;
}

template <typename R>
mcrt_status batch_tune(Batch& B, const mcrt_batch_cfg* c, LaunchShape& best, double* ms_tune) {
    const double t0 = now_ms();
    std::vector<LaunchShape> cand;
    for (int bs : {128, 256})
        for (int K : {2, 4, 8})
            for (int d : {8, 32}) {
                const int bpc = batch_max_blocks_per_cu<R>(K, B.layout, bs);
                cand.push_back({bs, K, d, bpc});
            }
    const double frac = c->tune_fraction > 0.0 ? c->tune_fraction : 0.02;
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    float best_ms = 1e30f;
    std::vector<uint32_t> keys(B.n());
    for (size_t t = 0; t < cand.size(); ++t) {
        for (int i = 0; i < B.n(); ++i) keys[i] = 0x40000000u | (uint32_t)t;
        mcrt_status r = batch_upload<R>(B, frac, 0, cand[t], keys);
        if (r == MCRT_OK) {
            hipEventRecord(e0, B.s);
            r = batch_pass_ops<R>(B, frac, cand[t], false, false, false);
            hipEventRecord(e1, B.s);
        }
        if (r != MCRT_OK) {
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return r;
        }
        hipEventSynchronize(e1);
        float ms = 0.f;
        hipEventElapsedTime(&ms, e0, e1);
        if (ms < best_ms) {
            best_ms = ms;
            best = cand[t];
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    *ms_tune = now_ms() - t0;
    return MCRT_OK;
}

template <typename R>
mcrt_status batch_run(Batch& B, const mcrt_batch_cfg* c, mcrt_batch_stats* st) {
    const double t0 = now_ms();
    // launch shape: explicit fields, else tuned (cached per workload class), else defaults
    LaunchShape sh{256, 4, 16, batch_max_blocks_per_cu<R>(4, B.layout, 256)};
    const bool explicit_shape = c->block_size > 0 && c->walk_batch > 0 && c->defer_lanes > 0;
    if (!explicit_shape && c->autotune) {
        int64_t cells = 0, packets = 0;
        for (mcrt_model* m : B.ms) {
            cells += m->ncell;
            packets += m->cfg.n_packets;
        }
        const auto key = std::make_tuple((int)B.f32, (int)lround(log2((double)cells)),
                                         (int)lround(log2((double)packets / (double)cells)));
        bool hit = false;
        {
            std::lock_guard<std::mutex> g(g_tune_mu);
            auto it = g_tune_cache.find(key);
            if (it != g_tune_cache.end()) {
                sh = it->second;
                hit = true;
            }
        }
        if (hit) {
            st->tuned = 2;
        } else {
            mcrt_status r = batch_tune<R>(B, c, sh, &st->ms_tune);
            if (r != MCRT_OK) return r;
            std::lock_guard<std::mutex> g(g_tune_mu);
            g_tune_cache[key] = sh;
            st->tuned = 1;
        }
    }
    if (c->block_size > 0) sh.block_size = c->block_size;
    if (c->walk_batch > 0) sh.walk_batch = c->walk_batch;
    if (c->defer_lanes > 0) sh.defer = c->defer_lanes;
    sh.bpc = c->blocks_per_cu > 0 ? c->blocks_per_cu
                                  : batch_max_blocks_per_cu<R>(sh.walk_batch, B.layout, sh.block_size);
    st->block_size = sh.block_size;
    st->walk_batch = sh.walk_batch;
    st->defer_lanes = sh.defer;
    st->blocks_per_cu = sh.bpc;

    // Lucy iterations
    const double ti = now_ms();
    std::vector<uint32_t> keys(B.n());
    for (int i = 0; i < B.n(); ++i) {
        mcrt_model* m = B.ms[i];
        keys[i] = (uint32_t)m->iter;
        mcrt_status r = set_weights(m, m->cfg.n_packets);
        if (r != MCRT_OK) return r;
    }
    mcrt_status r = batch_upload<R>(B, 1.0, 0, sh, keys);
    if (r != MCRT_OK) return r;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    for (int it = 0; it < c->n_iter; ++it) {
        const double t_it = now_ms();
        const bool replay = c->use_graph && it > 0;
        if (replay && !exec) {
            BCHK(hipStreamBeginCapture(B.s, hipStreamCaptureModeThreadLocal));
            r = batch_pass_ops<R>(B, 1.0, sh, true, true, true);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(B.s, &g);
            if (r != MCRT_OK) return r;
            BCHK(e);
            graph = g;
            BCHK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
            st->graph_used = 1;
        }
        if (replay) {
            BCHK(hipGraphLaunch(exec, B.s));
        } else {
            hipEventRecord(B.ms[0]->ev[0], B.s);
            r = batch_pass_ops<R>(B, 1.0, sh, false, false, false);
            if (r != MCRT_OK) return r;
            hipEventRecord(B.ms[0]->ev[1], B.s);
            for (mcrt_model* m : B.ms) {
                CellParams P;
                make_cell_params(m, P);
                BCHK(hipMemsetAsync(m->misc.p + MISC_STATS, 0, 8 * sizeof(unsigned long long), B.s));
                BCHK(launch_update(P, grid_blocks(m, m->ncell), B.s));
            }
            BCHK(launch_add_u32(B.n(), B.d_keys, 1u, 1, B.s));
        }
        BCHK(hipStreamSynchronize(B.s));
        if (!replay) {
            float ms = 0.f;
            hipEventElapsedTime(&ms, B.ms[0]->ev[0], B.ms[0]->ev[1]);
            st->ms_transport_last = ms;
        }
        for (mcrt_model* m : B.ms) {
            m->iter++;
            m->have_prev = 1;
        }
        st->n_iterations++;
        if (c->verbose) {
            fprintf(stderr, "# batch iteration %d of %d: %.1f ms%s\n", it + 1, c->n_iter, now_ms() - t_it,
                    replay ? " (graph replay)" : "");
            fflush(stderr);
        }
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    st->ms_iterations = now_ms() - ti;
    st->n_cross_dust = st->n_cross_empty = 0;
    for (mcrt_model* m : B.ms) {
        unsigned long long h[C_COUNT];
        BCHK(hipMemcpy(h, m->misc.p + MISC_CNT, sizeof h, hipMemcpyDeviceToHost));
        st->n_cross_dust += (int64_t)h[C_CROSS_DUST];
        st->n_cross_empty += (int64_t)h[C_CROSS_EMPTY];
        st->packets_per_iteration += m->cfg.n_packets;
    }

    // final binning pass
    if (c->final_pass) {
        const double tf = now_ms();
        for (int i = 0; i < B.n(); ++i) {
            mcrt_model* m = B.ms[i];
            keys[i] = 0x80000000u | (uint32_t)m->iter;
            const int64_t npf = m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets;
            r = set_weights(m, npf);
            if (r != MCRT_OK) return r;
            r = clear_bins(m);
            if (r != MCRT_OK) return r;
        }
        r = batch_upload<R>(B, 1.0, 1, sh, keys);
        if (r != MCRT_OK) return r;
        for (mcrt_model* m : B.ms) {
            const int64_t npf = m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets;
            r = prepare_pass(m, npf, false, true);
            if (r != MCRT_OK) return r;
        }
        BCHK(launch_fill_u64(1, B.pool(), 0ull, 1, B.s));
        int64_t total = 0;
        for (mcrt_model* m : B.ms)
            total += m->cfg.n_packets_final > 0 ? m->cfg.n_packets_final : m->cfg.n_packets;
        int64_t blocks = std::min<int64_t>((int64_t)B.n_cu * sh.bpc, (total + sh.block_size - 1) / sh.block_size);
        BCHK(launch_transport_batch<R>((const TransportParams<R>*)B.d_params, B.d_chunks, B.n(),
                                       B.pool(), B.d_keys, sh.walk_batch, B.layout,
                                       (int)std::max<int64_t>(blocks, 1), sh.block_size, B.s));
        BCHK(hipStreamSynchronize(B.s));
        st->ms_final = now_ms() - tf;
    }
    st->ms_total = now_ms() - t0;
    return MCRT_OK;
}

}  // namespace

extern "C" {

mcrt_status mcrt_batch_cfg_default(mcrt_batch_cfg* c) {
    if (!c) return MCRT_E_ARG;
    memset(c, 0, sizeof *c);
    c->n_iter = 5;
    c->final_pass = 1;
    c->use_graph = 1;
    c->autotune = 1;
    c->tune_fraction = 0.02;
    return MCRT_OK;
}

mcrt_status mcrt_batch_run(mcrt_model* const* models, int n, const mcrt_batch_cfg* c,
                           mcrt_batch_stats* st) {
    if (!models || n < 1 || !c || !st) return MCRT_E_ARG;
    for (int i = 0; i < n; ++i)
        if (!models[i]) return MCRT_E_ARG;
    memset(st, 0, sizeof *st);
    st->n_models = n;
    Batch B;
    B.ms.assign(models, models + n);
    mcrt_model* m0 = models[0];
    if (c->n_iter < 0 || c->block_size < 0 || c->block_size % 64 != 0 || c->block_size > 256 ||
        c->defer_lanes < 0 || c->defer_lanes > 64 || c->blocks_per_cu < 0)
        return fail(m0, MCRT_E_ARG, "bad batch configuration");
    if (c->walk_batch != 0 && c->walk_batch != 2 && c->walk_batch != 4 && c->walk_batch != 8)
        return fail(m0, MCRT_E_ARG, "batch walk_batch must be 2, 4 or 8");
    hipSetDevice(m0->device);
    B.f32 = m0->cfg.precision == MCRT_FP32_TRANSPORT;
    B.layout = m0->cfg.grid_layout == 1 ? 1 : 0;
    B.n_cu = m0->n_cu;
    B.s = m0->stream;
    for (int i = 0; i < n; ++i) {
        mcrt_model* m = models[i];
        if (m->device != m0->device) return fail(m0, MCRT_E_ARG, "batch models on different devices");
        if ((m->cfg.precision == MCRT_FP32_TRANSPORT) != B.f32 || (m->cfg.grid_layout == 1) != (B.layout == 1))
            return fail(m0, MCRT_E_ARG, "batch models differ in precision or grid layout");
        for (int j = 0; j < i; ++j)
            if (models[j] == m) return fail(m0, MCRT_E_ARG, "a model appears twice in the batch");
        mcrt_status r = ready(m);
        if (r != MCRT_OK) {
            if (m != m0) m0->err = "model " + std::to_string(i) + ": " + m->err;
            return r;
        }
    }
    // every model works on the batch stream for the duration of the call
    for (mcrt_model* m : B.ms) {
        hipStreamSynchronize(m->stream);
        B.saved_streams.push_back(m->stream);
        m->stream = B.s;
    }
    const size_t psz = B.f32 ? sizeof(TransportParams<float>) : sizeof(TransportParams<double>);
    if (hipMalloc(&B.d_params, psz * n) != hipSuccess ||
        hipMalloc((void**)&B.d_chunks, (n + 2) * sizeof(unsigned long long)) != hipSuccess ||
        hipMalloc((void**)&B.d_keys, n * sizeof(uint32_t)) != hipSuccess)
        return fail(m0, MCRT_E_NOMEM, "batch buffers");
    return B.f32 ? batch_run<float>(B, c, st) : batch_run<double>(B, c, st);
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Learned warm start: features of a model, and network -> starting T.
namespace mcrt {
namespace nn {
hipError_t launch_features(int64_t nvox, int nx, int ny, const double* rho, double chi1_dx,
                           const double* dep, const int* dcell, const double* dval, int nd, float* x,
                           hipStream_t st);
}  // namespace nn
}  // namespace mcrt

extern "C" {

mcrt_status mcrt_model_features(mcrt_model* m, float* d_x, size_t n) {
    if (!m || !d_x) return MCRT_E_ARG;
    if (!m->have_grid || !m->have_rho || !m->have_nu || !m->have_dust)
        return fail(m, MCRT_E_STATE, "set grid, density, frequencies and dust first");
    if ((int64_t)n != 3 * m->ncell) return fail(m, MCRT_E_SIZE, "features need 3 values per cell");
    hipSetDevice(m->device);
    // extinction of the bin holding 1 micron
    const double nu1 = 2.99792458e10 / 1e-4;
    const int nnu = (int)m->chi.size();
    int k = 0;
    while (k + 1 < nnu && m->nu[k + 1] <= nu1) ++k;
    const double dx = m->dx[0];
    // luminosity per cell; a source on a wall/edge/corner is shared by the touching cells
    std::vector<double> flux((size_t)m->ncell, 0.0);
    for (const Source& s : m->src) {
        int lo_i[3], hi_i[3];
        for (int a = 0; a < 3; ++a) {
            const double f = (s.pos[a] - m->lo[a]) / m->dx[a];
            const double fl = floor(f);
            int c = (int)fl;
            lo_i[a] = hi_i[a] = std::min(std::max(c, 0), m->n[a] - 1);
            if (f == fl && c > 0 && c < m->n[a]) lo_i[a] = c - 1;  // on an interior wall
        }
        const int cnt = (hi_i[0] - lo_i[0] + 1) * (hi_i[1] - lo_i[1] + 1) * (hi_i[2] - lo_i[2] + 1);
        const double share = s.lum / cnt / (4.0 * M_PI * dx * dx);
        for (int kk = lo_i[2]; kk <= hi_i[2]; ++kk)
            for (int j = lo_i[1]; j <= hi_i[1]; ++j)
                for (int i = lo_i[0]; i <= hi_i[0]; ++i)
                    flux[i + (size_t)m->n[0] * (j + (size_t)m->n[1] * kk)] += share;
    }
    std::vector<int> dcell;
    std::vector<double> dval;
    for (size_t j = 0; j < flux.size(); ++j)
        if (flux[j] > 0.0) {
            dcell.push_back((int)(j % m->n[0]));
            dcell.push_back((int)((j / m->n[0]) % m->n[1]));
            dcell.push_back((int)(j / ((size_t)m->n[0] * m->n[1])));
            dval.push_back(flux[j]);
        }
    const int nd = (int)dval.size();
    DBuf<double> dflux, ddval;
    DBuf<int> ddcell;
    HIPCHK(dflux.ensure(flux.size()));
    HIPCHK(ddval.ensure(nd > 0 ? nd : 1));
    HIPCHK(ddcell.ensure(nd > 0 ? 3 * nd : 3));
    HIPCHK(hipMemcpyAsync(dflux.p, flux.data(), flux.size() * sizeof(double), hipMemcpyHostToDevice,
                          m->stream));
    if (nd > 0) {
        HIPCHK(hipMemcpyAsync(ddval.p, dval.data(), nd * sizeof(double), hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(ddcell.p, dcell.data(), 3 * nd * sizeof(int), hipMemcpyHostToDevice,
                              m->stream));
    }
    HIPCHK(nn::launch_features(m->ncell, m->n[0], m->n[1], m->rho64.p, m->chi[k] * dx, dflux.p, ddcell.p,
                               ddval.p, nd, d_x, m->stream));
    HIPCHK(hipStreamSynchronize(m->stream));
    dflux.release();
    ddval.release();
    ddcell.release();
    return MCRT_OK;
}

mcrt_status mcrt_warm_start(mcrt_model* m, mcrt_surrogate* s, double* ms) {
    if (!m || !s) return MCRT_E_ARG;
    const double t0 = now_ms();
    if (!(m->n[0] == m->n[1] && m->n[1] == m->n[2]) || m->n[0] % 8 != 0)
        return fail(m, MCRT_E_ARG, "warm start needs a cubic grid with a side that is a multiple of 8");
    hipSetDevice(m->device);
    DBuf<float> x;
    DBuf<double> T;
    HIPCHK(x.ensure((size_t)3 * m->ncell));
    HIPCHK(T.ensure((size_t)m->ncell));
    mcrt_status r = mcrt_model_features(m, x.p, (size_t)3 * m->ncell);
    if (r == MCRT_OK) {
        r = mcrt_surrogate_predict_T(s, x.p, 1, m->n[0], T.p);
        if (r != MCRT_OK) m->err = std::string("surrogate: ") + mcrt_surrogate_last_error(s);
    }
    if (r == MCRT_OK) r = mcrt_set_temperature_device(m, T.p, 1, (size_t)m->ncell);
    x.release();
    T.release();
    if (ms) *ms = now_ms() - t0;
    return r;
}

}  // extern "C"
