// mcrt_internal.h -- parameter blocks shared by the host driver and the
// gfx950 kernels of libmcrt.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mcrt.h"

namespace mcrt {

constexpr int kRows = 128;          // emissivity rows, log-spaced in T over [1 K, 1e4 K]
constexpr double kTLo = 1.0;        // K
constexpr double kTHi = 1.0e4;      // K
constexpr int kRayTRows = 2048;     // rows of the raytracing table of ln B_k(ln T)
constexpr double kLnBFloor = -690.0; // ln B of a bin whose Planck integral underflows
constexpr double kTFloor = 1.0;     // K, temperature of cells that absorbed nothing
constexpr int kTSolveRows = 2048;   // rows of the ln Adot(ln T) table of the T solve
constexpr int kMrwRows = 2048;      // rows of the Planck/Rosseland mean table, log-spaced in T
constexpr int kMrwYRows = 8192;     // rows of the walk's first-passage inverse y(w), w = ln(u/(1-u))
constexpr double kMrwW0 = -37.5, kMrwW1 = 37.5;  // its range of w (|w| <= 36.8 for FP64 uniforms)
constexpr int kWave = 64;

// Per-lane counters flushed once per wave at the end of a transport launch.
enum CounterIdx { C_CROSS_DUST = 0, C_CROSS_EMPTY, C_SCATTER, C_ABSORB, C_ESCAPE, C_KILLED,
                  C_MRW, C_COUNT };

constexpr int kGroup = 16;          // CDF entries per group of the two-level search
constexpr int kPoolChunk = 64;      // packet ids a wave takes from the pool at a time

// Transport launch parameters (one model).  R is the transport precision.
template <typename R>
struct TransportParams {
    // grid
    int n[3];
    int bx, bxy;            // bricks along x, bricks per z layer (4x4x4 layout)
    double lo[3];
    double dx[3];           // cell size, cm
    R dxr[3];               // same in R
    R inv_dx[3];            // 1/dx in R
    const R* rho;           // [ncell or bricked] density in the transport layout
    // CDF tables are padded to npad = kGroup*ngroup entries per row (pad 2.0);
    // coarse[r*ngroup + q] = cdf[r*npad + kGroup*q + kGroup-1]
    int npad, ngroup;
    const R* ecoarse;       // [kRows*ngroup]
    const R* scoarse;       // [nsrc*ngroup]
    int lds_tables;         // stage lcdf, ecoarse, scoarse in LDS
    // dust per frequency bin
    int nnu;
    const R* chi;
    const R* kap;
    const R* alb;
    const R* g;
    // sources
    int nsrc;
    int sampling;           // 0 luminosity-proportional, 1 equal numbers
    const double* spos;     // [3*nsrc]
    const int4* scell;      // [nsrc] a source's cell (x, y, z) and w: bit a set when it lies
                            // on a cell wall of axis a (the direction's sign picks the cell)
    const double* sfrac;    // [3*nsrc] its offsets in that cell, in cells
    const R* lcdf;          // [nsrc] luminosity CDF
    const R* scdf;          // [nsrc*npad] spectral CDFs
    const double* sweight;  // [nsrc] packet weight relative to eps0 (equal sampling)
    // emission rows of every cell: position p in [0, kRows-1]; row m = floor(p), weight p-m
    const R* ecdf;          // [kRows*npad]
    const R* rowpos;        // [ncell] (x-fastest)
    // random numbers
    uint32_t key0, key1;
    // packets
    uint64_t n_packets;
    uint64_t packet_base;   // id of the first packet of this launch
    unsigned long long* pool;  // packets handed out so far (relative to packet_base)
    double eps0;            // erg per packet of weight 1
    int64_t max_events;
    int defer_lanes;
    // tallies (transport layout)
    double* acc;            // sum of weight * l * kappa over segments (cm^3 g^-1 per eps0)
    double* acc2;           // [ncell] sum of squares, or null
    size_t acc_stride;      // elements between the per-XCD copies of acc (0: one copy)
    int binning;
    int n_incl;
    double* sed_sum;
    double* sed_sum2;
    unsigned long long* sed_n;
    int n_img, npix;
    double img_hw;
    const int* img_of_bin;  // [nnu] image index or -1
    double* img_sum;
    double* img_sum2;
    // peeling-off (Sec. 2.6.2): n_peel observer unit vectors; SED
    // [n_peel][2][nnu] (0 direct, 1 scattered/re-emitted) and images
    // [n_img][n_peel][npix][npix], energy per steradian
    int n_peel;
    const double* peel_dir;  // [3*n_peel]
    const R* rho_lin;        // density x-fastest (the ray march to the boundary)
    // modified random walk (mrw_gamma 0 = off): cell temperatures (x-fastest)
    // and the table of kappa_P, d kappa_P / d ln T, chi_R, d chi_R / d ln T
    // per row of ln T over [kTLo, kTHi]
    double mrw_gamma;
    const double* Tcell;
    const double* mrw_tab;   // [kMrwRows * 4]
    const double* mrw_ytab;  // [kMrwYRows * 2]: y and dy/dw of the first-passage inverse against w = logit(u)
    double* psed_sum;
    double* psed_sum2;
    double* pimg_sum;
    double* pimg_sum2;
    // event log
    int64_t ev_packets;
    int ev_cap;
    mcrt_event* evlog;
    int32_t* evcount;
    // counters
    unsigned long long* counters;  // [C_COUNT]
    double* energies;              // [2] escaped, killed
};

// Raytracing of the emission toward the peel-off observers (FP64 throughout).
struct RayParams {
    int n[3];
    double lo[3], hi[3], dx[3];
    const double* rho;      // [ncell] density, x fastest
    const double* T;        // [ncell] temperature, K
    int nnu;
    const double* nu;       // [nnu+1] bin edges, Hz
    const double* chi;      // [nnu] extinction opacity, cm^2/g
    const double* kap;      // [nnu] absorption opacity, cm^2/g
    int n_obs;
    const double* dirs;     // [3*n_obs] unit vectors toward the observers
    int npix;
    double hw;              // image half width, cm
    int nsrc;
    const double* spos;     // [3*nsrc]
    const double* lsrc;     // [nsrc*nnu] source luminosity per bin, erg/s
    double* cube;           // [n_obs][npix][npix][nnu], erg/s/sr per pixel
    double* sed;            // [n_obs][2][nnu] (0 sources, 1 dust), erg/s/sr
    // ln B_k and d ln B_k / d ln T at ln T = ln kTLo + i dlnT (i < kRayTRows),
    // [row][bin] pairs; temperatures outside [kTLo, kTHi] use quadrature
    const double2* btab;
    double dlnT;
};

// Partial diffusion approximation: the grid, the selection inputs and the
// conjugate-gradient vectors (all [ncell], x-fastest).
struct PdaParams {
    int64_t ncell;
    int n[3];
    double dx[3];
    const double* rho;
    double* T;               // read; the connected PDA cells' T written at the end
    const double* adot;      // the Monte-Carlo estimate the selection uses
    const double* adot_sig;  // its error, or null
    double noise;            // relative error above which a cell is a PDA cell
    const double* mrw_tab;   // Rosseland mean table (kMrwRows x 4)
    const double* lnA;       // ln Adot(ln T) table and slopes (Eq. 3)
    const double* slope;
    double dy;
    unsigned char* flag;     // 0 not PDA, 1 PDA, 2 PDA connected to a sampled cell
    double *a, *x, *r, *z, *p, *q, *diag, *b;
    double* red;             // [5] r.z, p.q, new r.z, r.r, b.b
    unsigned* count;         // cells connected in a round
    double* adot_out;        // Adot of the connected PDA cells
    unsigned char* valid;
};

// Tiled sweeps: control words of a pass, in device memory.  Buffer b (0, 1)
// holds packet records; a sweep reads one buffer and writes the other.
struct SweepCtl {
    unsigned rec_alloc[2];        // record slots handed out in buffer b
    unsigned n_ent[2];            // entry slots handed out for buffer b
    unsigned item_next;           // work items taken in the current sweep
    unsigned n_items;             // work items of the current sweep
    unsigned overflow;            // a buffer or the entry list ran out of room
    unsigned done;                // no record left and every packet emitted
    unsigned sweeps;              // sweeps that walked records
    unsigned pad;
    unsigned long long emitted;   // packets emitted so far in this pass
    unsigned long long emit_first, emit_count;  // the refill of the current step
    unsigned long long visits;    // records walked (tile visits) so far
    unsigned drain;               // the pass's tail goes to the per-lane finish
    unsigned drain_buf;           // the buffer whose records it finishes
    unsigned drain_next;          // entries taken by the finish
    unsigned drain_recs;          // records it finishes
};

// Tiled sweeps: the tiling and the buffers of a pass.  A record's state is
// five (FP32) or nine (FP64) 16-byte quads; quad q of record i is at
// recs[b][q * cap + i].  Records are written in chunks of 64 slots per
// destination tile; every chunk (and every block of emitted packets of one
// tile) is registered as an entry (first record, count) of its tile, and the
// entries, grouped by tile, are the next sweep's work.
struct SweepParams {
    int txy;                    // tile extent in x and y (cells): 16 or 32
    int tz;                     // tile extent in z (cells)
    int ntx, nty, ntz, ntiles;  // tiles per axis, total
    // ceil(2^16 / txy), ceil(2^16 / tz): c / t = (c * m) >> 16 exactly for
    // cell coordinates c < 1024 and tile extents t <= 64
    unsigned mxy, mz;
    int visit_events;           // interactions per visit before a packet yields
    int item_ent;               // entries per work item
    int service;                // lanes of a wave that wait before its events and exits run
    unsigned cap;               // record slots per buffer
    unsigned max_ent;           // entries per buffer
    uint4* recs[2];
    unsigned* ent_tile[2];      // tile of each registered entry
    uint2* ent[2];              // (first record, count) of each registered entry
    uint2* sent;                // the entries of the buffer being read, grouped by tile
    unsigned* tile_rec;         // [ntiles] records registered per tile
    unsigned* tile_ent;         // [ntiles] entries registered per tile
    unsigned* ent_off;          // [ntiles+1] first grouped entry of each tile
    uint4* item_desc;           // per work item: tile, first grouped entry, entry count, 1
    unsigned* cursor;           // [ntiles] grouping cursors
    SweepCtl* ctl;
    unsigned long long n_packets;  // packets of the pass
    unsigned long long batch;      // refill batch
    unsigned long long drain_below;  // finish per lane once at most this many records remain (0: never)
};

// Cell-update parameters (always FP64).
struct CellParams {
    int64_t ncell;
    int n[3];
    int brick;              // acc/acc2 are in the 4x4x4 brick layout
    int bx, bxy;
    double eps_over_vol;    // eps0 / (Delta t V), Delta t = 1 s
    const double* rho;
    const double* acc;
    int acc_copies;         // copies of acc to sum, acc_stride elements apart
    size_t acc_stride;
    const double* acc2;     // or null
    double* adot;
    double* adot_prev;
    double* adot_sig;
    double* T;
    double* T_prev;
    double* sig_rel;
    double* sig_rel_prev;
    unsigned char* valid;       // T came from a sampled cell or from the user
    unsigned char* valid_prev;
    const double* lnA;      // [kTSolveRows] ln Adot at ln T = i*dy
    const double* slope;    // [kTSolveRows] dlnAdot/dlnT
    double dy;
    int have_prev;          // Adot of the previous iteration exists
    int want_noise;
    double noise_thres;
    double* Rbuf;           // [ncell] R_j or +inf
    double* rbuf;           // [ncell] r_j or +inf
    unsigned long long* stats;  // [8] n_r, n_mask, n_unsampled, n_clamped, max_r bits
};

}  // namespace mcrt
