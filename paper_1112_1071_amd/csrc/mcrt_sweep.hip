// mcrt_sweep.hip -- tiled transport: packets grouped by grid tile, each tile
// walked with its density and absorption tally staged in LDS.
//
// The grid is cut into tiles of txy x txy x tz cells.  A pass runs in sweeps.
// Between sweeps every packet in flight is a record in global memory (its
// full state: cell, direction, flight origin, wall distances, ray distance,
// sampled and used optical depth, weight, bin, event counts and the position
// in its random stream), and the records are grouped by the tile the packet
// is in.  In a sweep, a workgroup takes work items (each up to S.item
// records of one tile); for each new tile it loads the tile's density into
// LDS and clears an LDS tally, and its lanes walk the item's packets
// (Sec. 2.2; Lucy's path-length estimator, Sec. 2.3 Eq. 2, added into the
// LDS tally) until each leaves the tile, escapes the grid, is
// killed, or has had visit_events interactions in this visit; a packet that
// leaves (or yields) is written out with the tile it is now in.  When the
// workgroup moves on to another tile (or ends), it adds the LDS tally into
// the FP64 global tally, one atomic per touched cell of the tile.  Sweeps
// repeat until no packet is left.
//
// Every packet follows the same arithmetic, random numbers and decisions as
// in the per-lane persistent kernel (the walk is the same segment by segment,
// only cut at tile walls); tallies differ only in summation order (and, in
// the FP32 form, in summing a visit's contributions in FP32 before the FP64
// flush).
#include <math.h>

#include "mcrt_internal.h"
#include "mcrt_packet.h"

namespace mcrt {

constexpr int kDrainEvents = 32;     // interactions per visit once an item is drained
constexpr unsigned kNoTile = 0xffffffffu;  // tile of a hole in the records (no packet)
constexpr int kEmitHistTiles = 16384;      // tiles counted in LDS by the emission (64 KB)
enum : int { ST_MOVE = 5, ST_YIELD = 6 };

// State of a packet between visits (the Packet fields that are not
// recomputed from the direction, the bin and the stream position).
template <typename R> struct __attribute__((aligned(16))) PacketRec {
    int c0, c1, c2, k;
    R d0, d1, d2, u0, u1, u2, tx, ty, tz, t, tau, tau_acc, wgt;
    uint32_t nev, nlog, n, st;
    uint64_t id;
};

__device__ __forceinline__ int tile_of(const SweepParams& S, int c0, int c1, int c2) {
    return (c0 / S.txy) + S.ntx * ((c1 / S.txy) + S.nty * (c2 / S.tz));
}

template <typename R>
__device__ __forceinline__ void store_rec(PacketRec<R>* r, const Packet<R>& s, const Stream<R>& rs,
                                          int st) {
    PacketRec<R> q;
    q.c0 = s.c0;
    q.c1 = s.c1;
    q.c2 = s.c2;
    q.k = s.k;
    q.d0 = s.d0;
    q.d1 = s.d1;
    q.d2 = s.d2;
    q.u0 = s.u0;
    q.u1 = s.u1;
    q.u2 = s.u2;
    q.tx = s.tx;
    q.ty = s.ty;
    q.tz = s.tz;
    q.t = s.t;
    q.tau = s.tau;
    q.tau_acc = s.tau_acc;
    q.wgt = s.wgt;
    q.nev = s.nev;
    q.nlog = s.nlog;
    q.n = rs.n;
    q.st = (uint32_t)st;
    q.id = s.id;
    *r = q;
}

template <typename R>
__device__ __forceinline__ void unpack_rec(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                           const PacketRec<R>& q, const R* chi_t, const R* kap_t) {
    s.c0 = q.c0;
    s.c1 = q.c1;
    s.c2 = q.c2;
    s.k = q.k;
    s.d0 = q.d0;
    s.d1 = q.d1;
    s.d2 = q.d2;
    s.u0 = q.u0;
    s.u1 = q.u1;
    s.u2 = q.u2;
    s.tx = q.tx;
    s.ty = q.ty;
    s.tz = q.tz;
    s.t = q.t;
    s.tau = q.tau;
    s.tau_acc = q.tau_acc;
    s.wgt = q.wgt;
    s.nev = q.nev;
    s.nlog = q.nlog;
    s.id = q.id;
    s.st = (int)q.st;
    // the same quotients begin_flight computed for this flight
    s.dtx = P.dxr[0] / fabs(s.d0);
    s.dty = P.dxr[1] / fabs(s.d1);
    s.dtz = P.dxr[2] / fabs(s.d2);
    s.chi = chi_t[s.k];
    s.kap = kap_t[s.k];
    const uint64_t gid = P.packet_base + s.id;
    rs.p0 = (uint32_t)gid;
    rs.p1 = (uint32_t)(gid >> 32);
    rs.n = q.n;
    if (rs.n & 1u) {  // the second uniform of the last Philox call is still unused
        uint32_t c0 = rs.n >> 1, c1 = 0u, c2 = rs.p0, c3 = rs.p1;
        philox4x32_10(c0, c1, c2, c3, rs.k0, rs.k1);
        rs.s0 = c2;
        rs.s1 = c3;
    }
}

// Local LDS index of the packet's cell in the tile with origin (o0, o1, o2).
__device__ __forceinline__ int tile_index(int c0, int c1, int c2, int o0, int o1, int o2, int txy) {
    return (c0 - o0) + txy * ((c1 - o1) + txy * (c2 - o2));
}

// Up to K segments of the walk inside the tile with origin (o0, o1, o2):
// segment by segment the arithmetic of walk(), with density and tally in LDS.
// The segments are written without branches (a lane that stopped keeps its
// values through selects), so that a wave runs straight-line code; the one
// division, for the segment that ends in an interaction, is taken after the
// loop.  The lane carries its cell's LDS index jl and density rho between
// calls (an interaction leaves the cell unchanged); the next cell's density
// is read as soon as the next cell is known, ahead of the segment's arithmetic.
// Cell coordinates are not stepped per segment: each axis counts the moves
// left before the packet reaches the last cell of the tile (or of the grid,
// in a ragged tile) in its direction, and the coordinates follow from the
// counts after the loop.  A crossing with no move left on its axis leaves the
// tile (state MOVE, into the neighbour tile's cell) or, at the grid's own
// wall, the grid (state ESC, the cell unchanged).
template <typename R, int K, bool NOISE>
__device__ __forceinline__ void walk_tile(Packet<R>& s, const TransportParams<R>& P, int o0, int o1,
                                          int o2, int txy, int tz, const R* __restrict__ rho_t,
                                          R* __restrict__ acc_t, double* __restrict__ acc2_t,
                                          uint32_t* cnt, int& jl, R& rho) {
    const bool px = s.d0 > (R)0, py = s.d1 > (R)0, pz = s.d2 > (R)0;
    const int sx = px ? 1 : -1;
    const int sy = py ? 1 : -1;
    const int sz = pz ? 1 : -1;
    const int djy = sy * txy, djz = sz * txy * txy;
    // one past the last cell of the tile that lies in the grid, per axis
    const int h0 = min(o0 + txy, P.n[0]), h1 = min(o1 + txy, P.n[1]), h2 = min(o2 + tz, P.n[2]);
    const int r0i = px ? h0 - 1 - s.c0 : s.c0 - o0;
    const int r1i = py ? h1 - 1 - s.c1 : s.c1 - o1;
    const int r2i = pz ? h2 - 1 - s.c2 : s.c2 - o2;
    int r0 = r0i, r1 = r1i, r2 = r2i;  // moves left inside the tile per axis
    bool act = true;    // still walking in this call
    bool hit = false;   // the last segment ends in an interaction
    bool left = false;  // the last segment crosses the tile's (or grid's) wall
    int lax = 0;        // and on which axis
    R rc_h = (R)1, ts_h = (R)0;
    int jl_h = jl;
    uint32_t nd = 0, ne = 0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool ax1 = s.ty < s.tx;
        R tm = ax1 ? s.ty : s.tx;
        const bool ax2 = s.tz < tm;
        tm = ax2 ? s.tz : tm;
        const int r = ax2 ? r2 : (ax1 ? r1 : r0);
        const bool edge = r == 0;  // the next cell is outside the tile or the grid
        const int dj = ax2 ? djz : (ax1 ? djy : sx);
        const int jn = edge ? jl : jl + dj;
        const R rho_n = rho_t[jn];
        // this segment
        const R ts = s.t;
        const R l = fmax(tm - s.t, (R)0);
        const bool dust = rho > (R)0;
        const R rc = rho * s.chi;
        const R dtau = rc * l;
        const bool h = act && dust && s.tau_acc + dtau >= s.tau;
        const bool cross = act && !h;  // the segment reaches the cell wall
        nd += (act && dust) ? 1u : 0u;
        ne += (act && !dust) ? 1u : 0u;
        if (h) {
            hit = true;
            rc_h = rc;
            ts_h = ts;
            jl_h = jl;
        }
        if (cross && dust) {
            s.tau_acc += dtau;
            const R w = s.wgt * l * s.kap;
            atomicAdd(acc_t + jl, w);
            if (NOISE) atomicAdd(acc2_t + jl, (double)w * (double)w);  // w^2 may exceed FP32
        }
        s.t = cross ? fmax(tm, s.t) : s.t;
        const bool mv = cross && !edge;
        const bool m0 = mv && !ax1 && !ax2, m1 = mv && ax1 && !ax2, m2 = mv && ax2;
        r0 -= m0 ? 1 : 0;
        r1 -= m1 ? 1 : 0;
        r2 -= m2 ? 1 : 0;
        s.tx += m0 ? s.dtx : (R)0;
        s.ty += m1 ? s.dty : (R)0;
        s.tz += m2 ? s.dtz : (R)0;
        const bool lv = cross && edge;
        left = left || lv;
        lax = lv ? (ax2 ? 2 : (ax1 ? 1 : 0)) : lax;
        act = mv;
        jl = mv ? jn : jl;
        rho = mv ? rho_n : rho;
    }
    s.c0 += sx * (r0i - r0);
    s.c1 += sy * (r1i - r1);
    s.c2 += sz * (r2i - r2);
    int st = ST_WALK;
    if (hit) {
        const R l = (s.tau - s.tau_acc) / rc_h;
        const R w = s.wgt * l * s.kap;
        atomicAdd(acc_t + jl_h, w);
        if (NOISE) atomicAdd(acc2_t + jl_h, (double)w * (double)w);
        s.t = ts_h + l;
        st = ST_EVENT;
    } else if (left) {
        // past the tile's wall on axis lax: the neighbour tile's cell, or out
        // of the grid if that wall is the grid's
        const int c = lax == 0 ? s.c0 : (lax == 1 ? s.c1 : s.c2);
        const int sg = lax == 0 ? sx : (lax == 1 ? sy : sz);
        const int g = lax == 0 ? P.n[0] : (lax == 1 ? P.n[1] : P.n[2]);
        if ((unsigned)(c + sg) >= (unsigned)g) {
            st = ST_ESC;
        } else {
            st = ST_MOVE;
            if (lax == 0) {
                s.c0 += sx;
                s.tx += s.dtx;
            } else if (lax == 1) {
                s.c1 += sy;
                s.ty += s.dty;
            } else {
                s.c2 += sz;
                s.tz += s.dtz;
            }
        }
    }
    s.st = st;
    cnt[C_CROSS_DUST] += nd;
    cnt[C_CROSS_EMPTY] += ne;
}

// Append the lanes' records whose state is ST_MOVE or ST_YIELD (one atomic per
// wave) and free those lanes.  Returns the record's tile in dest (or -1).
template <typename R>
__device__ __forceinline__ void append_moves(const SweepParams& S, Packet<R>& s, const Stream<R>& rs,
                                             int lane, int& dest) {
    dest = -1;
    const bool mine = s.st == ST_MOVE || s.st == ST_YIELD;
    const unsigned long long mv = __ballot(mine);
    if (!mv) return;
    const int leader = __ffsll((long long)mv) - 1;
    unsigned base = 0;
    if (lane == leader) base = atomicAdd(S.out_count, (unsigned)__popcll(mv));
    base = __shfl(base, leader);
    if (mine) {
        const unsigned idx = base + (unsigned)__popcll(mv & __lanemask_lt());
        store_rec(reinterpret_cast<PacketRec<R>*>(S.out) + idx, s, rs,
                  s.st == ST_YIELD ? ST_EVENT : ST_WALK);
        dest = tile_of(S, s.c0, s.c1, s.c2);
        S.out_tile[idx] = (unsigned)dest;
        s.st = ST_EMPTY;
    }
}

// count records per destination tile: one global atomic per distinct tile of
// the wave
__device__ __forceinline__ void count_tiles(unsigned* counts, int dest) {
    bool pending = dest >= 0;
    for (;;) {
        const unsigned long long act = __ballot(pending);
        if (!act) break;
        const int leader = __ffsll((long long)act) - 1;
        const int lt = __shfl(dest, leader);
        const bool mine = pending && dest == lt;
        const unsigned long long same = __ballot(mine);
        if (__lane_id() == leader) atomicAdd(counts + lt, (unsigned)__popcll(same));
        if (mine) pending = false;
    }
}

template <typename R>
__device__ __forceinline__ void flush_block_counters(const TransportParams<R>& P, uint32_t* cnt,
                                                     double e_escaped, double e_killed,
                                                     unsigned long long* s_cnt, double* s_energy) {
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) atomicAdd(&s_cnt[c], (unsigned long long)cnt[c]);
    atomicAdd(&s_energy[0], e_escaped);
    atomicAdd(&s_energy[1], e_killed);
    __syncthreads();
    if (threadIdx.x < C_COUNT) atomicAdd(P.counters + threadIdx.x, s_cnt[threadIdx.x]);
    if (threadIdx.x < 2) unsafeAtomicAdd(P.energies + threadIdx.x, s_energy[threadIdx.x]);
}

// Emission of packets [first, first+count): each starts its first flight
// (exactly as in the per-lane kernel) and is written as record base+i with its
// tile; a packet that starts outside the grid escapes at once (or is killed by
// the modified random walk at the event limit) and leaves a hole
// (tile kNoTile, skipped by the ordering).  Positions need no atomics; the
// per-tile counts are gathered in an LDS histogram per block when the tiles
// fit (hist), else per wave.
template <typename R>
__global__ void __launch_bounds__(256) k_sweep_emit(TransportParams<R> P, SweepParams S,
                                                     uint64_t first, uint64_t count, unsigned base,
                                                     int hist) {
    extern __shared__ unsigned s_hist[];
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    if (hist)
        for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) s_hist[t] = 0u;
    __syncthreads();
    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    const Tables<R> tb{P.lcdf, P.ecoarse, P.scoarse};
    Stream<R> rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.n = 0;
    rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    PacketRec<R>* out = reinterpret_cast<PacketRec<R>*>(S.out);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t b0 = (uint64_t)blockIdx.x * blockDim.x; b0 < count; b0 += stride) {
        const uint64_t i = b0 + threadIdx.x;
        int dest = -1;
        if (i < count) {
            Packet<R> s;
            emit(s, rs, P, tb, first + i, cnt, e_killed, global_deposit<0>(P, P.acc));
            const unsigned idx = base + (unsigned)i;
            if (s.st == ST_ESC || s.st == ST_EMPTY) {  // escaped at once, or killed by the walk
                if (s.st == ST_ESC) escape(s, P, cnt, e_escaped);
                S.out_tile[idx] = kNoTile;
            } else {
                store_rec(out + idx, s, rs, ST_WALK);
                dest = tile_of(S, s.c0, s.c1, s.c2);
                S.out_tile[idx] = (unsigned)dest;
                if (hist) atomicAdd(&s_hist[dest], 1u);
            }
        }
        if (!hist) count_tiles(S.counts, dest);
    }
    if (hist) {
        __syncthreads();
        for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x)
            if (s_hist[t]) atomicAdd(S.counts + t, s_hist[t]);
    }
    flush_block_counters(P, cnt, e_escaped, e_killed, s_cnt, s_energy);
}

// The tile's counts of records written for it and its face neighbours, and its
// LDS partial sums into the FP64 tally (cells of this tile only); the LDS is
// free again on return.
template <typename R>
__device__ __forceinline__ void flush_tile(const TransportParams<R>& P, const SweepParams& S, int tile,
                                           int o0, int o1, int o2, int txy, int tcells,
                                           const R* acc_t, const double* acc2_t, unsigned* s_nb) {
    __syncthreads();
    if (threadIdx.x < 7 && s_nb[threadIdx.x]) {
        const int off[7] = {0, -1, 1, -S.ntx, S.ntx, -S.ntx * S.nty, S.ntx * S.nty};
        atomicAdd(S.counts + tile + off[threadIdx.x], s_nb[threadIdx.x]);
    }
    for (int i = threadIdx.x; i < tcells; i += blockDim.x) {
        const R a = acc_t[i];
        const double a2 = acc2_t ? acc2_t[i] : 0.0;
        if (a != (R)0 || a2 != 0.0) {
            const int lx = i % txy, ly = (i / txy) % txy, lz = i / (txy * txy);
            const int64_t j = (o0 + lx) + (int64_t)P.n[0] * ((o1 + ly) + (int64_t)P.n[1] * (o2 + lz));
            if (a != (R)0) unsafeAtomicAdd(P.acc + j, (double)a);
            if (a2 != 0.0) unsafeAtomicAdd(P.acc2 + j, a2);
        }
    }
    __syncthreads();
    if (threadIdx.x < 7) s_nb[threadIdx.x] = 0u;
}

// One sweep over the work items (persistent workgroups; in FP32 of up to 512
// threads, so that one group of 8 waves can hold a 32x32x16 tile, 128 KB of
// LDS; the FP64 walk keeps its registers at 256 threads).
template <typename R, int K>
__global__ void __launch_bounds__(sizeof(R) == 4 ? 512 : 256) k_sweep(TransportParams<R> P, SweepParams S) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ unsigned s_item, s_next;
    __shared__ unsigned s_nb[7];  // records leaving for this tile, -x, +x, -y, +y, -z, +z
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    const int txy = S.txy;
    const int tcells = txy * txy * S.tz;
    // LDS: Sum w^2 (FP64, when kept), density, tally, staged tables
    double* acc2_t = P.acc2 ? reinterpret_cast<double*>(smem_raw) : nullptr;
    R* rho_t = reinterpret_cast<R*>(smem_raw + (P.acc2 ? tcells * sizeof(double) : 0));
    R* acc_t = rho_t + tcells;
    R* chi_t = acc_t + tcells;  // bin opacities
    R* kap_t = chi_t + P.nnu;
    R* sm_tab = kap_t + P.nnu;
    for (int i = threadIdx.x; i < P.nnu; i += blockDim.x) {
        chi_t[i] = P.chi[i];
        kap_t[i] = P.kap[i];
    }
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    Tables<R> tb;
    if (P.lds_tables) {
        const int ne = kRows * P.ngroup, ns = P.nsrc * P.ngroup;
        for (int i = threadIdx.x; i < P.nsrc; i += blockDim.x) sm_tab[i] = P.lcdf[i];
        for (int i = threadIdx.x; i < ne; i += blockDim.x) sm_tab[P.nsrc + i] = P.ecoarse[i];
        for (int i = threadIdx.x; i < ns; i += blockDim.x) sm_tab[P.nsrc + ne + i] = P.scoarse[i];
        tb.lcdf = sm_tab;
        tb.ecoarse = sm_tab + P.nsrc;
        tb.scoarse = sm_tab + P.nsrc + ne;
    } else {
        tb.lcdf = P.lcdf;
        tb.ecoarse = P.ecoarse;
        tb.scoarse = P.scoarse;
    }
    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    const int lane = __lane_id();
    const int defer = P.defer_lanes;
    const PacketRec<R>* in = reinterpret_cast<const PacketRec<R>*>(S.in);
    Stream<R> rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.n = 0;
    rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    const unsigned n_items = S.item_off[S.ntiles];
    if (threadIdx.x < 7) s_nb[threadIdx.x] = 0u;
    int tile = -1;  // the tile held in LDS (block-uniform)
    int o0 = 0, o1 = 0, o2 = 0;

    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(S.item_next, 1u);
        __syncthreads();
        const unsigned item = s_item;
        if (item >= n_items) break;
        int lo = 0, hi = S.ntiles - 1;  // last tile whose first item is <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (S.item_off[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        if (lo != tile) {
            // an item of the tile already in LDS keeps it; otherwise the tile
            // in LDS goes out before the item's tile comes in
            if (tile >= 0) flush_tile(P, S, tile, o0, o1, o2, txy, tcells, acc_t, acc2_t, s_nb);
            tile = lo;
            const int tzi = tile / (S.ntx * S.nty);
            const int trem = tile - tzi * S.ntx * S.nty;
            const int tyi = trem / S.ntx, txi = trem - tyi * S.ntx;
            o0 = txi * txy;
            o1 = tyi * txy;
            o2 = tzi * S.tz;
            for (int i = threadIdx.x; i < tcells; i += blockDim.x) {
                const int lx = i % txy, ly = (i / txy) % txy, lz = i / (txy * txy);
                const int gx = o0 + lx, gy = o1 + ly, gz = o2 + lz;
                R r = (R)0;
                if (gx < P.n[0] && gy < P.n[1] && gz < P.n[2])
                    r = P.rho[gx + (int64_t)P.n[0] * (gy + (int64_t)P.n[1] * gz)];
                rho_t[i] = r;
                acc_t[i] = (R)0;
                if (acc2_t) acc2_t[i] = 0.0;
            }
        }
        if (threadIdx.x == 0) s_next = 0u;
        __syncthreads();
        const unsigned first = S.tile_off[tile] + (item - S.item_off[tile]) * S.item;
        const unsigned end = min(first + S.item, S.tile_off[tile + 1]);

        Packet<R> s;
        s.st = ST_EMPTY;
        int jl = 0;       // the packet's cell in LDS
        R rho = (R)0;     // and its density
        int visit = 0;
        bool drained = false;  // this item's records are all taken (wave-uniform)
        for (;;) {
            const unsigned long long need = __ballot(s.st == ST_EMPTY);
            if (need) {
                const int leader = __ffsll((long long)need) - 1;
                unsigned base = 0;
                if (lane == leader) base = atomicAdd(&s_next, (unsigned)__popcll(need));
                base = __shfl(base, leader);
                if (s.st == ST_EMPTY) {
                    const unsigned slot = first + base + (unsigned)__popcll(need & __lanemask_lt());
                    if (slot < end) {
                        unpack_rec(s, rs, P, in[S.order[slot]], chi_t, kap_t);
                        jl = tile_index(s.c0, s.c1, s.c2, o0, o1, o2, txy);
                        rho = rho_t[jl];
                        visit = 0;
                        // a record is always mid-walk or at a pending event
                        if (s.st != ST_WALK && s.st != ST_EVENT) s.st = ST_DONE;
                    } else {
                        s.st = ST_DONE;
                    }
                }
            }
            if (__ballot(s.st != ST_DONE) == 0ull) break;
            drained = drained || __ballot(s.st == ST_DONE) != 0ull;
            for (;;) {
                if (s.st == ST_WALK) {
                    // Sum w^2 is kept (the tally's noise estimate) or not for the whole launch
                    if (acc2_t)
                        walk_tile<R, K, true>(s, P, o0, o1, o2, txy, S.tz, rho_t, acc_t, acc2_t, cnt, jl, rho);
                    else
                        walk_tile<R, K, false>(s, P, o0, o1, o2, txy, S.tz, rho_t, acc_t, nullptr, cnt, jl, rho);
                }
                if (__ballot(s.st == ST_WALK) == 0ull) break;
                if (__popcll(__ballot(s.st != ST_WALK && s.st != ST_DONE)) >= defer) break;
            }
            if (s.st == ST_EVENT) {
                // a packet yields (back to this tile's queue for the next sweep)
                // after visit_events interactions in this visit, or after
                // kDrainEvents once the item is drained, so that no workgroup
                // waits long on one random walk; every visit makes progress
                // (a crossing of the tile wall, an escape, or an interaction)
                const int cap = drained && S.visit_events > kDrainEvents ? kDrainEvents : S.visit_events;
                if (visit >= cap) {
                    s.st = ST_YIELD;
                } else {
                    ++visit;
                    interact(s, rs, P, tb, cnt, e_killed, TileDeposit<R>{acc_t, acc2_t, o0, o1, o2, txy});
                }
            }
            if (s.st == ST_ESC) escape(s, P, cnt, e_escaped);
            int dest;
            append_moves(S, s, rs, lane, dest);
            if (dest >= 0) {
                int nb = 0;  // a packet moves at most one cell: this tile or a face neighbour
                const int dt = dest - tile;
                if (dt == -1) nb = 1;
                else if (dt == 1) nb = 2;
                else if (dt == -S.ntx) nb = 3;
                else if (dt == S.ntx) nb = 4;
                else if (dt == -S.ntx * S.nty) nb = 5;
                else if (dt == S.ntx * S.nty) nb = 6;
                atomicAdd(&s_nb[nb], 1u);
            }
        }
    }
    if (tile >= 0) flush_tile(P, S, tile, o0, o1, o2, txy, tcells, acc_t, acc2_t, s_nb);
    flush_block_counters(P, cnt, e_escaped, e_killed, s_cnt, s_energy);
}

// ---- grouping the written records by tile ---------------------------------
// (the counts per tile were taken while the records were written)

// exclusive scans of the counts (records and work items), cursors, and the
// counters of the next sweep; one block
__global__ void __launch_bounds__(1024) k_tile_scan(unsigned* __restrict__ counts, int ntiles,
                                                    unsigned kItem,
                                                    unsigned* __restrict__ tile_off,
                                                    unsigned* __restrict__ item_off,
                                                    unsigned* __restrict__ cursor,
                                                    unsigned* __restrict__ item_next) {
    __shared__ unsigned s_a[1024], s_b[1024];
    const int per = (ntiles + (int)blockDim.x - 1) / (int)blockDim.x;
    const int t0 = threadIdx.x * per;
    unsigned ra = 0, rb = 0;
    for (int t = t0; t < t0 + per && t < ntiles; ++t) {
        ra += counts[t];
        rb += (counts[t] + kItem - 1) / kItem;
    }
    s_a[threadIdx.x] = ra;
    s_b[threadIdx.x] = rb;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const unsigned va = threadIdx.x >= (unsigned)o ? s_a[threadIdx.x - o] : 0u;
        const unsigned vb = threadIdx.x >= (unsigned)o ? s_b[threadIdx.x - o] : 0u;
        __syncthreads();
        s_a[threadIdx.x] += va;
        s_b[threadIdx.x] += vb;
        __syncthreads();
    }
    unsigned pa = s_a[threadIdx.x] - ra, pb = s_b[threadIdx.x] - rb;  // exclusive
    for (int t = t0; t < t0 + per && t < ntiles; ++t) {
        const unsigned c = counts[t];
        tile_off[t] = pa;
        cursor[t] = pa;
        item_off[t] = pb;
        pa += c;
        pb += (c + kItem - 1) / kItem;
        counts[t] = 0u;
    }
    if (threadIdx.x == blockDim.x - 1) {
        tile_off[ntiles] = s_a[threadIdx.x];
        item_off[ntiles] = s_b[threadIdx.x];
        *item_next = 0u;
    }
}

// order[cursor[tile]++] = record index.  A block takes kOrderChunk consecutive
// records (written by a few hundred waves, so they fall into few tiles), counts
// them per tile in an LDS hash table, reserves each tile's range with one global
// atomic, and places every record at its reserved base + its rank in the block.
// A record whose tile finds no free hash slot takes its position directly.
constexpr int kOrderChunk = 4096;
constexpr int kOrderHash = 1024;

__global__ void __launch_bounds__(256) k_tile_order(const unsigned* __restrict__ out_tile,
                                                    const unsigned* __restrict__ n_out,
                                                    unsigned* __restrict__ cursor,
                                                    unsigned* __restrict__ order) {
    __shared__ unsigned h_key[kOrderHash], h_cnt[kOrderHash];
    constexpr int per = kOrderChunk / 256;
    const unsigned n = *n_out;
    for (unsigned c0 = blockIdx.x * (unsigned)kOrderChunk; c0 < n; c0 += gridDim.x * (unsigned)kOrderChunk) {
        for (int i = threadIdx.x; i < kOrderHash; i += blockDim.x) {
            h_key[i] = 0xffffffffu;
            h_cnt[i] = 0u;
        }
        __syncthreads();
        int slot[per];
        unsigned rank[per];
#pragma unroll
        for (int j = 0; j < per; ++j) {
            const unsigned i = c0 + (unsigned)(j * 256) + threadIdx.x;
            slot[j] = -1;
            rank[j] = 0u;
            const unsigned t = i < n ? out_tile[i] : kNoTile;
            if (t != kNoTile) {
                unsigned h = (t * 2654435761u) >> 22;
                int found = -1;
                for (int probe = 0; probe < kOrderHash; ++probe) {
                    const unsigned k = atomicCAS(&h_key[h], 0xffffffffu, t);
                    if (k == 0xffffffffu || k == t) {
                        found = (int)h;
                        break;
                    }
                    h = (h + 1u) & (kOrderHash - 1);
                }
                if (found >= 0) {
                    slot[j] = found;
                    rank[j] = atomicAdd(&h_cnt[found], 1u);
                } else {
                    order[atomicAdd(cursor + t, 1u)] = i;  // table full
                }
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kOrderHash; e += blockDim.x)
            if (h_cnt[e]) h_cnt[e] = atomicAdd(cursor + h_key[e], h_cnt[e]);  // count -> base
        __syncthreads();
#pragma unroll
        for (int j = 0; j < per; ++j)
            if (slot[j] >= 0) order[h_cnt[slot[j]] + rank[j]] = c0 + (unsigned)(j * 256) + threadIdx.x;
        __syncthreads();
    }
}

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
size_t sweep_record_bytes(int fp32) {
    return fp32 ? sizeof(PacketRec<float>) : sizeof(PacketRec<double>);
}

template <typename R> using SweepFn = void (*)(TransportParams<R>, SweepParams);

template <typename R> SweepFn<R> pick_sweep(int K) {
    switch (K) {
        case 1: return k_sweep<R, 1>;
        case 2: return k_sweep<R, 2>;
        default: return k_sweep<R, 4>;
    }
}

template <typename R>
hipError_t launch_sweep_emit(const TransportParams<R>& P, const SweepParams& S, uint64_t first,
                             uint64_t count, unsigned base, int blocks, hipStream_t st) {
    const int hist = S.ntiles <= kEmitHistTiles ? 1 : 0;
    hipLaunchKernelGGL(k_sweep_emit<R>, dim3(blocks), dim3(256), hist ? S.ntiles * sizeof(unsigned) : 0, st,
                       P, S, first, count, base, hist);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sweep(const TransportParams<R>& P, const SweepParams& S, int K, int blocks,
                        int threads, size_t lds, hipStream_t st) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(pick_sweep<R>(K)),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(pick_sweep<R>(K), dim3(blocks), dim3(threads), lds, st, P, S);
    return hipGetLastError();
}

template <typename R> int sweep_max_blocks_per_cu(int K, int threads, size_t lds) {
    int nb = 0;
    if (lds > 65536)
        hipFuncSetAttribute(reinterpret_cast<const void*>(pick_sweep<R>(K)),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_sweep<R>(K), threads, lds) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

hipError_t launch_tile_sort(const SweepParams& S, unsigned* order, unsigned* tile_off,
                            unsigned* item_off, unsigned* cursor, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, S.counts, S.ntiles, S.item, tile_off,
                       item_off, cursor, S.item_next);
    hipLaunchKernelGGL(k_tile_order, dim3(blocks), dim3(256), 0, st, S.out_tile, S.out_count, cursor,
                       order);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0,
                       st, p, n, v);
    return hipGetLastError();
}

template hipError_t launch_sweep_emit<float>(const TransportParams<float>&, const SweepParams&,
                                             uint64_t, uint64_t, unsigned, int, hipStream_t);
template hipError_t launch_sweep_emit<double>(const TransportParams<double>&, const SweepParams&,
                                              uint64_t, uint64_t, unsigned, int, hipStream_t);
template hipError_t launch_sweep<float>(const TransportParams<float>&, const SweepParams&, int, int,
                                        int, size_t, hipStream_t);
template hipError_t launch_sweep<double>(const TransportParams<double>&, const SweepParams&, int,
                                         int, int, size_t, hipStream_t);
template int sweep_max_blocks_per_cu<float>(int, int, size_t);
template int sweep_max_blocks_per_cu<double>(int, int, size_t);

}  // namespace mcrt
