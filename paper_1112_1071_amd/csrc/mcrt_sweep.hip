// mcrt_sweep.hip -- tiled transport: packets grouped by grid tile, each tile
// walked with its density and absorption tally staged in LDS.
//
// The grid is cut into tiles of txy x txy x tz cells.  A pass runs in sweeps.
// Between sweeps every packet in flight is a record in one of two buffers:
// its full state (cell, direction, flight origin, wall distances, ray
// distance, sampled and used optical depth, weight, bin, event counts, the
// position in its random stream), stored as 16-byte quads in planes, so that
// the 64 lanes of a wave that read consecutive records load 1 KB contiguous
// per quad.  Records are written in chunks of 64 slots per destination tile
// (each wave keeps one open chunk per neighbour of the tile it walks); a
// full chunk, and the rest of a chunk when the wave moves to another tile, is
// registered as an entry (first record, count) of its tile.  Between sweeps
// the entries are grouped by tile (a counting sort of the entries, not of the
// records) and cut into work items.
//
// In a sweep a workgroup takes work items (up to item_ent entries of one
// tile); for each new tile it loads the tile's density into LDS and clears an
// LDS tally.  Its waves take the item's entries one at a time and hand their
// records to lanes; each lane holds the packet it walks and the record of the
// packet it walks next, loaded while the current one walks.  A lane walks its
// packet (Sec. 2.2; Lucy's path-length estimator, Sec. 2.3 Eq. 2, added into
// the LDS tally) until it leaves the tile, escapes the grid, is killed, or has
// had visit_events interactions in this visit; interactions, escapes and
// exits of a wave are handled together once `service` of its lanes wait.  A
// packet that leaves (or yields) is written to the chunk of the tile it is
// now in.  When the workgroup moves to another tile (or ends), it adds the LDS
// tally into the FP64 global tally, one atomic per touched cell.
//
// The sweeps of a pass run without a host round trip: a one-thread kernel
// decides on the device whether to refill the pool (emit the next batch of
// packets when fewer than `batch` records are in flight), the emission writes
// its packets as records of their start tiles, a one-block kernel scans the
// per-tile counts, and the entries are grouped before the sweep reads them.
//
// Every packet follows the same arithmetic, random numbers and decisions as
// in the per-lane persistent kernel (the walk is the same segment by segment,
// only cut at tile walls); tallies differ only in summation order (and, in
// the FP32 form, in summing a visit's contributions in FP32 before the FP64
// flush).
#include <math.h>

#include <type_traits>

#include "mcrt_internal.h"
#include "mcrt_packet.h"

namespace mcrt {

constexpr int kDrainEvents = 32;     // interactions per visit once an item is drained
constexpr unsigned kChunk = 64;      // record slots per chunk
constexpr unsigned kNone = 0xffffffffu;
constexpr int kEmitPer = 16;         // packets per thread of an emission step
constexpr int kEmitThreads = 256;
constexpr int kEmitStep = kEmitPer * kEmitThreads;  // packets per block and step
constexpr int kEmitHash = 1024;      // tiles an emission block counts in LDS
constexpr int kMaxItemEnt = 256;     // entries of a work item (the host keeps item_ent below)
enum : int { ST_MOVE = 5, ST_YIELD = 6 };
enum : unsigned { RS_WALK = 0u, RS_EVENT = 1u, RS_HOLE = 2u };  // record states

// ---- records ----------------------------------------------------------------
template <typename R> struct Rec;
template <> struct Rec<float> { static constexpr int NQ = 5; };
template <> struct Rec<double> { static constexpr int NQ = 9; };
template <typename R> struct Raw { uint4 q[Rec<R>::NQ]; };

__device__ __forceinline__ uint32_t pack_cell(int c0, int c1, int c2, unsigned rs) {
    return (uint32_t)c0 | ((uint32_t)c1 << 10) | ((uint32_t)c2 << 20) | (rs << 30);
}
__device__ __forceinline__ uint32_t f2u(float x) { return __float_as_uint(x); }
__device__ __forceinline__ float u2f(uint32_t x) { return __uint_as_float(x); }
__device__ __forceinline__ uint2 d2u(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return make_uint2((uint32_t)b, (uint32_t)(b >> 32));
}
__device__ __forceinline__ double u2d(uint32_t lo, uint32_t hi) {
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ uint4 dd2q(double a, double b) {
    const uint2 x = d2u(a), y = d2u(b);
    return make_uint4(x.x, x.y, y.x, y.y);
}

__device__ __forceinline__ void pack_rec(Raw<float>& r, const Packet<float>& s, const Stream<float>& rs,
                                         unsigned state) {
    r.q[0] = make_uint4(pack_cell(s.c0, s.c1, s.c2, state), (uint32_t)s.k, s.nev, rs.n);
    r.q[1] = make_uint4(f2u(s.d0), f2u(s.d1), f2u(s.d2), f2u(s.t));
    r.q[2] = make_uint4(f2u(s.u0), f2u(s.u1), f2u(s.u2), f2u(s.tau));
    r.q[3] = make_uint4(f2u(s.tx), f2u(s.ty), f2u(s.tz), f2u(s.tau_acc));
    r.q[4] = make_uint4((uint32_t)s.id, (uint32_t)(s.id >> 32), f2u(s.wgt), s.nlog);
}
__device__ __forceinline__ void pack_rec(Raw<double>& r, const Packet<double>& s, const Stream<double>& rs,
                                         unsigned state) {
    r.q[0] = make_uint4(pack_cell(s.c0, s.c1, s.c2, state), (uint32_t)s.k, s.nev, rs.n);
    r.q[1] = dd2q(s.d0, s.d1);
    r.q[2] = dd2q(s.d2, s.t);
    r.q[3] = dd2q(s.u0, s.u1);
    r.q[4] = dd2q(s.u2, s.tau);
    r.q[5] = dd2q(s.tx, s.ty);
    r.q[6] = dd2q(s.tz, s.tau_acc);
    r.q[7] = make_uint4((uint32_t)s.id, (uint32_t)(s.id >> 32), s.nlog, 0u);
    r.q[8] = dd2q(s.wgt, 0.0);
}

// record state RS_* of a raw record
template <typename R> __device__ __forceinline__ unsigned rec_state(const Raw<R>& r) { return r.q[0].x >> 30; }

__device__ __forceinline__ void unpack_fields(Packet<float>& s, uint32_t& n, const Raw<float>& r) {
    s.k = (int)r.q[0].y;
    s.nev = r.q[0].z;
    n = r.q[0].w;
    s.d0 = u2f(r.q[1].x); s.d1 = u2f(r.q[1].y); s.d2 = u2f(r.q[1].z); s.t = u2f(r.q[1].w);
    s.u0 = u2f(r.q[2].x); s.u1 = u2f(r.q[2].y); s.u2 = u2f(r.q[2].z); s.tau = u2f(r.q[2].w);
    s.tx = u2f(r.q[3].x); s.ty = u2f(r.q[3].y); s.tz = u2f(r.q[3].z); s.tau_acc = u2f(r.q[3].w);
    s.id = (uint64_t)r.q[4].x | ((uint64_t)r.q[4].y << 32);
    s.wgt = u2f(r.q[4].z);
    s.nlog = r.q[4].w;
}
__device__ __forceinline__ void unpack_fields(Packet<double>& s, uint32_t& n, const Raw<double>& r) {
    s.k = (int)r.q[0].y;
    s.nev = r.q[0].z;
    n = r.q[0].w;
    s.d0 = u2d(r.q[1].x, r.q[1].y); s.d1 = u2d(r.q[1].z, r.q[1].w);
    s.d2 = u2d(r.q[2].x, r.q[2].y); s.t = u2d(r.q[2].z, r.q[2].w);
    s.u0 = u2d(r.q[3].x, r.q[3].y); s.u1 = u2d(r.q[3].z, r.q[3].w);
    s.u2 = u2d(r.q[4].x, r.q[4].y); s.tau = u2d(r.q[4].z, r.q[4].w);
    s.tx = u2d(r.q[5].x, r.q[5].y); s.ty = u2d(r.q[5].z, r.q[5].w);
    s.tz = u2d(r.q[6].x, r.q[6].y); s.tau_acc = u2d(r.q[6].z, r.q[6].w);
    s.id = (uint64_t)r.q[7].x | ((uint64_t)r.q[7].y << 32);
    s.nlog = r.q[7].z;
    s.wgt = u2d(r.q[8].x, r.q[8].y);
}

template <typename R>
__device__ __forceinline__ void store_raw(const SweepParams& S, uint4* recs, unsigned idx, const Raw<R>& r) {
#pragma unroll
    for (int q = 0; q < Rec<R>::NQ; ++q) recs[(size_t)q * S.cap + idx] = r.q[q];
}

template <typename R>
__device__ __forceinline__ void load_raw(const SweepParams& S, const uint4* recs, unsigned idx, Raw<R>& r) {
#pragma unroll
    for (int q = 0; q < Rec<R>::NQ; ++q) r.q[q] = recs[(size_t)q * S.cap + idx];
}

// The packet of a record: the state fields, then what begin_flight derived
// from them (wall spacings along the ray, the bin's opacities) and the random
// stream's position.
template <typename R>
__device__ __forceinline__ void unpack_rec(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                           const Raw<R>& r, const R* chi_t, const R* kap_t) {
    const uint32_t cw = r.q[0].x;
    s.c0 = (int)(cw & 1023u);
    s.c1 = (int)((cw >> 10) & 1023u);
    s.c2 = (int)((cw >> 20) & 1023u);
    const unsigned state = cw >> 30;
    if (state == RS_HOLE) {
        s.st = ST_EMPTY;
        return;
    }
    uint32_t n;
    unpack_fields(s, n, r);
    s.dtx = P.dxr[0] / fabs(s.d0);
    s.dty = P.dxr[1] / fabs(s.d1);
    s.dtz = P.dxr[2] / fabs(s.d2);
    s.chi = chi_t[s.k];
    s.kap = kap_t[s.k];
    const uint64_t gid = P.packet_base + s.id;
    rs.p0 = (uint32_t)gid;
    rs.p1 = (uint32_t)(gid >> 32);
    rs.n = n;
    // the second words of the last block are recomputed when drawn (most
    // visits draw nothing)
    rs.s0 = rs.s1 = 0u;
    s.st = state == RS_WALK ? ST_WALK : ST_EVENT;
}

// ---- tiles --------------------------------------------------------------------
// The tile of cell (c0, c1, c2); the quotients by the tile extents as
// multiplications by their rounded-up 2^16 reciprocals (exact for the
// extents and coordinates tiled sweeps allow).
__device__ __forceinline__ int tile_of(const SweepParams& S, int c0, int c1, int c2) {
    const int q0 = (int)(__umul24((unsigned)c0, S.mxy) >> 16);
    const int q1 = (int)(__umul24((unsigned)c1, S.mxy) >> 16);
    const int q2 = (int)(__umul24((unsigned)c2, S.mz) >> 16);
    return q0 + S.ntx * (q1 + S.nty * q2);
}

// the tile of destination slot d of tile t: itself, then -x, +x, -y, +y, -z, +z
__device__ __forceinline__ int slot_tile(const SweepParams& S, int t, int d) {
    const int nxy = S.ntx * S.nty;
    switch (d) {
        case 1: return t - 1;
        case 2: return t + 1;
        case 3: return t - S.ntx;
        case 4: return t + S.ntx;
        case 5: return t - nxy;
        case 6: return t + nxy;
        default: return t;
    }
}

// Global index of cell (c0, c1, c2).  Tiled sweeps hold at most 1024 cells
// per axis, so every factor fits 24 bits and the index 30.
template <typename R>
__device__ __forceinline__ unsigned grid_index(const TransportParams<R>& P, int c0, int c1, int c2) {
    return (unsigned)c0 +
           __umul24((unsigned)P.n[0], (unsigned)c1 + __umul24((unsigned)P.n[1], (unsigned)c2));
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
                                          double* __restrict__ acc_t, double* __restrict__ acc2_t,
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
    // moves left inside the tile per axis, ten bits each (a tile spans at
    // most 1023 cells per axis)
    uint32_t rp = (uint32_t)r0i | ((uint32_t)r1i << 10) | ((uint32_t)r2i << 20);
    bool act = true;    // still walking in this call
    bool hit = false;   // the last segment ends in an interaction
    bool left = false;  // the last segment crosses the tile's (or grid's) wall
    int lax = 0;        // and on which axis
    uint32_t nd = 0, ne = 0;
    const R wk = s.wgt * s.kap;  // tally weight per unit path length
#pragma unroll
    for (int i = 0; i < K; ++i) {
        const bool ax1 = s.ty < s.tx;
        R tm = ax1 ? s.ty : s.tx;
        const bool ax2 = s.tz < tm;
        tm = ax2 ? s.tz : tm;
        const uint32_t sh = ax2 ? 20u : (ax1 ? 10u : 0u);
        const bool edge = ((rp >> sh) & 1023u) == 0u;  // the next cell is outside the tile or the grid
        const int dj = ax2 ? djz : (ax1 ? djy : sx);
        const int jn = edge ? jl : jl + dj;
        const R rho_n = rho_t[jn];
        // this segment
        const R l = fmax(tm - s.t, (R)0);
        const bool dust = rho > (R)0;
        const R rc = rho * s.chi;
        const R dtau = rc * l;
        const bool h = act && dust && s.tau_acc + dtau >= s.tau;
        const bool cross = act && !h;  // the segment reaches the cell wall
        nd += (act && dust) ? 1u : 0u;
        ne += (act && !dust) ? 1u : 0u;
        // after an interaction nothing moves: the ray parameter, the cell and
        // its density stay those of the interaction's segment
        hit = hit || h;
        if (cross && dust) {
            s.tau_acc += dtau;
            const R w = wk * l;
            atomicAdd(acc_t + jl, (double)w);
            if (NOISE) atomicAdd(acc2_t + jl, (double)w * (double)w);  // w^2 may exceed FP32
        }
        // the ray parameter never decreases (a select: fmax would canonicalise
        // both operands on every segment)
        s.t = (cross && tm > s.t) ? tm : s.t;
        const bool mv = cross && !edge;
        const bool m0 = mv && !ax1 && !ax2, m1 = mv && ax1 && !ax2, m2 = mv && ax2;
        rp -= mv ? (1u << sh) : 0u;
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
    s.c0 += sx * (r0i - (int)(rp & 1023u));
    s.c1 += sy * (r1i - (int)((rp >> 10) & 1023u));
    s.c2 += sz * (r2i - (int)(rp >> 20));
    int st = ST_WALK;
    if (hit) {
        const R l = (s.tau - s.tau_acc) / (rho * s.chi);
        const R w = wk * l;
        atomicAdd(acc_t + jl, (double)w);
        if (NOISE) atomicAdd(acc2_t + jl, (double)w * (double)w);
        s.t = s.t + l;
        st = ST_EVENT;
        // the cell's emission row, loaded now for the interaction (an
        // absorption re-emits from it) while the wave walks on
        s.rowp = P.rowpos[grid_index(P, s.c0, s.c1, s.c2)];
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

// ---- entries and record slots -------------------------------------------------
// A sweep's records and entries are handed out from two counters per buffer.
// To keep atomics on those two addresses rare, a wave takes record slots
// kArenaSlots at a time and entry slots kArenaEnt at a time and hands them
// out itself; the per-tile record and entry counts of a workgroup's
// registrations are summed in LDS and added to the global counts when the
// workgroup leaves the tile.  Entry slots a wave still holds when the sweep
// ends are marked empty (count 0).
constexpr unsigned kArenaSlots = 1024;  // record slots a wave takes at a time (a multiple of kChunk)
constexpr unsigned kArenaEnt = 32;      // entry slots a wave takes at a time

// One wave's output state: its open chunk per destination slot of the tile it
// walks, and the record and entry slots it holds.
struct WaveOut {
    unsigned base[7];
    unsigned fill[7];
    unsigned rb, rl;  // record slots [rb, rb + rl)
    unsigned eb, el;  // entry slots [eb, eb + el)
};

__device__ __forceinline__ void wave_out_init(WaveOut& w) {
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        w.base[d] = kNone;
        w.fill[d] = 0u;
    }
    w.rb = w.rl = w.eb = w.el = 0u;
}

// kChunk record slots of buffer b (kNone when the buffer is full); wave-uniform
__device__ __forceinline__ unsigned take_chunk(const SweepParams& S, int b, WaveOut& w, int lane) {
    if (w.rl < kChunk) {
        unsigned f = 0u;
        if (lane == 0) {
            f = atomicAdd(&S.ctl->rec_alloc[b], kArenaSlots);
            if (f > S.cap || S.cap - f < kArenaSlots) {
                atomicOr(&S.ctl->overflow, 1u);
                f = kNone;
            }
        }
        f = (unsigned)__shfl((int)f, 0);
        if (f == kNone) return kNone;
        w.rb = f;
        w.rl = kArenaSlots;
    }
    const unsigned c = w.rb;
    w.rb += kChunk;
    w.rl -= kChunk;
    return c;
}

// Register records [first, first + count) as an entry of the tile in
// destination slot d; s_tc holds the workgroup's per-slot record and entry
// counts of the current tile.  Wave-uniform arguments.
__device__ __forceinline__ void wave_register(const SweepParams& S, int b, WaveOut& w, int tile, int d,
                                              unsigned first, unsigned count, unsigned* s_tc, int lane) {
    if (w.el == 0u) {
        unsigned e = 0u;
        if (lane == 0) {
            e = atomicAdd(&S.ctl->n_ent[b], kArenaEnt);
            if (e > S.max_ent || S.max_ent - e < kArenaEnt) {
                atomicOr(&S.ctl->overflow, 1u);
                e = kNone;
            }
        }
        e = (unsigned)__shfl((int)e, 0);
        if (e == kNone) return;
        w.eb = e;
        w.el = kArenaEnt;
    }
    if (lane == 0) {
        S.ent_tile[b][w.eb] = (unsigned)tile;
        S.ent[b][w.eb] = make_uint2(first, count);
        atomicAdd(&s_tc[2 * d], count);
        atomicAdd(&s_tc[2 * d + 1], 1u);
    }
    w.eb += 1u;
    w.el -= 1u;
}

// Emission: registration of a run of records of one tile in entry slot e.
__device__ __forceinline__ void emit_register(const SweepParams& S, int b, unsigned e, int tile, unsigned first,
                                              unsigned count) {
    S.ent_tile[b][e] = (unsigned)tile;
    S.ent[b][e] = make_uint2(first, count);
    atomicAdd(S.tile_rec + tile, count);
    atomicAdd(S.tile_ent + tile, 1u);
}

// Emission: n record slots (or entry slots, ent = true) of buffer b from the
// buffer's counter, kNone when the buffer is full.
__device__ __forceinline__ unsigned emit_take(const SweepParams& S, int b, unsigned n, bool ent) {
    unsigned* ctr = ent ? &S.ctl->n_ent[b] : &S.ctl->rec_alloc[b];
    const unsigned lim = ent ? S.max_ent : S.cap;
    const unsigned f = atomicAdd(ctr, n);
    if (f > lim || lim - f < n) {
        atomicOr(&S.ctl->overflow, 1u);
        return kNone;
    }
    return f;
}

// The entry slots a wave still holds are marked empty.
__device__ __forceinline__ void wave_out_release(const SweepParams& S, int b, WaveOut& w, int lane) {
    if ((unsigned)lane < w.el) S.ent[b][w.eb + lane] = make_uint2(0u, 0u);
    w.el = 0u;
}

// Register the wave's partly filled chunks (the wave leaves tile t).
__device__ __forceinline__ void chunks_close(const SweepParams& S, int b, int t, WaveOut& w, unsigned* s_tc,
                                             int lane) {
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        if (w.base[d] != kNone && w.fill[d] > 0u)
            wave_register(S, b, w, slot_tile(S, t, d), d, w.base[d], w.fill[d], s_tc, lane);
        w.base[d] = kNone;
        w.fill[d] = 0u;
    }
}

// The workgroup's per-slot counts of tile t into the global per-tile counts
// (threads 0..6, after a barrier that follows the last registration).
__device__ __forceinline__ void flush_tile_counts(const SweepParams& S, int t, unsigned* s_tc) {
    if (threadIdx.x < 7) {
        const int d = threadIdx.x;
        if (s_tc[2 * d]) atomicAdd(S.tile_rec + slot_tile(S, t, d), s_tc[2 * d]);
        if (s_tc[2 * d + 1]) atomicAdd(S.tile_ent + slot_tile(S, t, d), s_tc[2 * d + 1]);
        s_tc[2 * d] = 0u;
        s_tc[2 * d + 1] = 0u;
    }
}

// Write the records of the lanes whose packets leave the tile or yield
// (state MOVE / YIELD) into the open chunks of their destination tiles, and
// free those lanes.  Per destination: the wave's lanes take consecutive slots
// (their rank among the lanes of that destination); a chunk that fills is
// registered and the rest goes to a new chunk.  A packet that leaves has
// crossed one wall of the tile (origin o0, o1, o2) by one cell, so its
// destination slot follows from comparisons with the tile's bounds.
template <typename R>
__device__ __forceinline__ void write_exits(const SweepParams& S, int b, int tile, int o0, int o1, int o2,
                                            Packet<R>& s, const Stream<R>& rs, WaveOut& w, unsigned* s_tc,
                                            int lane) {
    const bool out = s.st == ST_MOVE || s.st == ST_YIELD;
    if (__ballot(out) == 0ull) return;
    const int slot = !out                    ? -1
                     : s.c0 < o0             ? 1
                     : s.c0 >= o0 + S.txy    ? 2
                     : s.c1 < o1             ? 3
                     : s.c1 >= o1 + S.txy    ? 4
                     : s.c2 < o2             ? 5
                     : s.c2 >= o2 + S.tz     ? 6
                                             : 0;
    unsigned idx = kNone;
#pragma unroll
    for (int d = 0; d < 7; ++d) {
        const unsigned long long m = __ballot(slot == d);
        if (m == 0ull) continue;
        const unsigned n = (unsigned)__popcll(m);
        const unsigned room = w.base[d] == kNone ? 0u : kChunk - w.fill[d];
        const unsigned k1 = n < room ? n : room;
        const unsigned nb = n > k1 ? take_chunk(S, b, w, lane) : kNone;
        if (slot == d) {
            const unsigned rank = (unsigned)__popcll(m & __lanemask_lt());
            if (rank < k1) idx = w.base[d] + w.fill[d] + rank;
            else idx = nb == kNone ? kNone : nb + (rank - k1);
        }
        if (w.base[d] != kNone && w.fill[d] + k1 == kChunk) {
            wave_register(S, b, w, slot_tile(S, tile, d), d, w.base[d], kChunk, s_tc, lane);
            w.base[d] = kNone;
            w.fill[d] = 0u;
        } else {
            w.fill[d] += k1;
        }
        if (n > k1) {
            w.base[d] = nb;
            w.fill[d] = nb == kNone ? 0u : n - k1;
        }
    }
    if (out) {
        if (idx != kNone) {
            Raw<R> r;
            pack_rec(r, s, rs, s.st == ST_YIELD ? RS_EVENT : RS_WALK);
            store_raw(S, S.recs[b], idx, r);
        }
        s.st = ST_EMPTY;
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

// ---- sweep control --------------------------------------------------------------
// The refill of this step: when fewer than batch records were registered for
// buffer b (summed over the tiles) and packets remain, the next batch is
// emitted into b.  One block.
__global__ void __launch_bounds__(1024) k_refill_plan(SweepParams S, int b) {
    __shared__ unsigned long long s_sum[1024];
    unsigned long long v = 0ull;
    for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) v += S.tile_rec[t];
    s_sum[threadIdx.x] = v;
    __syncthreads();
    for (int o = (int)blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s_sum[threadIdx.x] += s_sum[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        SweepCtl* c = S.ctl;
        unsigned long long cnt = 0ull;
        if (s_sum[0] < S.batch && c->emitted < S.n_packets) {
            const unsigned long long left = S.n_packets - c->emitted;
            cnt = left < S.batch ? left : S.batch;
        }
        c->emit_first = c->emitted;
        c->emit_count = cnt;
        c->emitted += cnt;
    }
}

// Emission of the step's refill into buffer b.  A block takes kEmitStep
// packets at a time: it first finds every packet's start tile (the first
// part of an emission: the same draws and arithmetic), counts them per tile in
// an LDS hash table, reserves one run of slots per tile and registers it as an
// entry; then it emits the packets in full and writes each at its tile's run
// plus its rank.  A packet that starts outside the grid escapes at once; one
// the modified random walk kills at emission leaves a hole in its run.  A tile
// that finds no free hash slot takes one slot and one entry per packet.
template <typename R, bool FULL>
__global__ void __launch_bounds__(kEmitThreads) k_sweep_emit(TransportParams<R> P, SweepParams S, int b) {
    __shared__ unsigned h_key[kEmitHash], h_cnt[kEmitHash], h_base[kEmitHash], h_ent[kEmitHash];
    __shared__ unsigned s_rtot, s_etot, s_rbase, s_ebase;
    __shared__ int s_slot[kEmitStep];  // per packet: hash slot, -1 own entry, -2 outside / none
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    const unsigned long long first = S.ctl->emit_first, count = S.ctl->emit_count;
    if (count == 0ull) return;
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    const Tables<R> tb = global_tables(P);
    Stream<R> rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.n = 0;
    rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    for (unsigned long long c0 = (unsigned long long)blockIdx.x * kEmitStep; c0 < count;
         c0 += (unsigned long long)gridDim.x * kEmitStep) {
        for (int i = threadIdx.x; i < kEmitHash; i += blockDim.x) {
            h_key[i] = kNone;
            h_cnt[i] = 0u;
        }
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < kEmitPer; ++j) {
            const unsigned long long i = c0 + (unsigned long long)(j * kEmitThreads) + threadIdx.x;
            int& slot = s_slot[j * kEmitThreads + threadIdx.x];
            slot = -2;  // no packet, or it starts outside the grid
            if (i < count) {
                int e0, e1, e2;
                emit_start_cell(rs, P, tb, first + i, e0, e1, e2);
                if (in_grid(P, e0, e1, e2)) {
                    const unsigned t = (unsigned)tile_of(S, e0, e1, e2);
                    unsigned h = (t * 2654435761u) >> 22;
                    slot = -1;  // no hash slot: one entry of its own
                    for (int probe = 0; probe < kEmitHash; ++probe) {
                        const unsigned k = atomicCAS(&h_key[h], kNone, t);
                        if (k == kNone || k == t) {
                            slot = (int)h;
                            atomicAdd(&h_cnt[h], 1u);
                            break;
                        }
                        h = (h + 1u) & (kEmitHash - 1);
                    }
                }
            }
        }
        // one run of slots per tile, one entry per run: the block's records and
        // entries are taken from the buffer's counters at once
        if (threadIdx.x == 0) {
            s_rtot = 0u;
            s_etot = 0u;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kEmitHash; e += blockDim.x) {
            h_base[e] = kNone;
            if (h_cnt[e]) {
                h_base[e] = atomicAdd(&s_rtot, h_cnt[e]);  // offset within the block's run
                h_ent[e] = atomicAdd(&s_etot, 1u);
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            s_rbase = s_rtot ? emit_take(S, b, s_rtot, false) : kNone;
            s_ebase = s_etot ? emit_take(S, b, s_etot, true) : kNone;
        }
        __syncthreads();
        for (int e = threadIdx.x; e < kEmitHash; e += blockDim.x) {
            if (h_cnt[e]) {
                if (s_rbase == kNone || s_ebase == kNone) {
                    h_base[e] = kNone;
                } else {
                    h_base[e] += s_rbase;
                    emit_register(S, b, s_ebase + h_ent[e], (int)h_key[e], h_base[e], h_cnt[e]);
                }
                h_cnt[e] = 0u;  // ranks from here on
            }
        }
        __syncthreads();
#pragma unroll 1
        for (int j = 0; j < kEmitPer; ++j) {
            const unsigned long long i = c0 + (unsigned long long)(j * kEmitThreads) + threadIdx.x;
            if (i >= count) continue;
            const int slot = s_slot[j * kEmitThreads + threadIdx.x];
            Packet<R> s;
            emit<R, GlobalDeposit<0>, FULL>(s, rs, P, tb, first + i, cnt, e_killed,
                                            global_deposit<0>(P, P.acc));
            if (slot == -2) {  // outside the grid: escapes at once
                if (s.st == ST_ESC) escape<R, FULL>(s, P, cnt, e_escaped);
                continue;
            }
            unsigned idx;
            if (slot >= 0) {
                const unsigned rank = atomicAdd(&h_cnt[slot], 1u);
                idx = h_base[slot] == kNone ? kNone : h_base[slot] + rank;
            } else {
                idx = emit_take(S, b, 1u, false);
                const unsigned e = idx == kNone ? kNone : emit_take(S, b, 1u, true);
                if (e != kNone) emit_register(S, b, e, tile_of(S, s.c0, s.c1, s.c2), idx, 1u);
                else idx = kNone;
            }
            if (idx == kNone) continue;
            Raw<R> r;
            pack_rec(r, s, rs, s.st == ST_WALK ? RS_WALK : RS_HOLE);
            store_raw(S, S.recs[b], idx, r);
        }
        __syncthreads();
    }
    flush_block_counters(P, cnt, e_escaped, e_killed, s_cnt, s_energy);
}

// Exclusive scans of the per-tile entry counts (grouped entry offsets), the
// work items of the sweep about to run, the grouping cursors, the sweep's
// statistics, and the reset of the counters of the buffer it writes; one
// block.  A tile's entries form items of item_ent entries and one item of
// the rest.  The sweep claims items in order, so they are listed longest
// first: all full items (tile by tile), then the remainders by decreasing
// size (a counting sort on the size), so that a sweep ends on short items
// and its groups finish close together.
__global__ void __launch_bounds__(1024) k_sweep_scan(SweepParams S, int b) {
    __shared__ unsigned s_a[1024], s_b[1024], s_r[1024];
    __shared__ unsigned s_hist[kMaxItemEnt], s_roff[kMaxItemEnt];
    if (S.ctl->drain) return;  // the tail went to the per-lane finish
    const int n = S.ntiles;
    const unsigned ie = (unsigned)S.item_ent;
    const int per = (n + (int)blockDim.x - 1) / (int)blockDim.x;
    const int t0 = threadIdx.x * per;
    for (int i = threadIdx.x; i < kMaxItemEnt; i += blockDim.x) s_hist[i] = 0u;
    __syncthreads();
    unsigned ra = 0, rb = 0, rr = 0;
    for (int t = t0; t < t0 + per && t < n; ++t) {
        const unsigned e = S.tile_ent[t];
        ra += e;
        rb += e / ie;  // full items
        rr += S.tile_rec[t];
        if (e % ie) atomicAdd(&s_hist[e % ie], 1u);
    }
    s_a[threadIdx.x] = ra;
    s_b[threadIdx.x] = rb;
    s_r[threadIdx.x] = rr;
    __syncthreads();
    for (int o = 1; o < (int)blockDim.x; o <<= 1) {
        const unsigned va = threadIdx.x >= (unsigned)o ? s_a[threadIdx.x - o] : 0u;
        const unsigned vb = threadIdx.x >= (unsigned)o ? s_b[threadIdx.x - o] : 0u;
        const unsigned vr = threadIdx.x >= (unsigned)o ? s_r[threadIdx.x - o] : 0u;
        __syncthreads();
        s_a[threadIdx.x] += va;
        s_b[threadIdx.x] += vb;
        s_r[threadIdx.x] += vr;
        __syncthreads();
    }
    const unsigned n_full = s_b[blockDim.x - 1];
    if (threadIdx.x == 0) {
        // remainder items after the full ones, the largest first
        unsigned o = n_full;
        for (int r = (int)ie - 1; r >= 1; --r) {
            s_roff[r] = o;
            o += s_hist[r];
        }
        s_roff[0] = o;  // the number of items
    }
    __syncthreads();
    unsigned pa = s_a[threadIdx.x] - ra, pb = s_b[threadIdx.x] - rb;  // exclusive
    for (int t = t0; t < t0 + per && t < n; ++t) {
        const unsigned e = S.tile_ent[t];
        S.ent_off[t] = pa;
        S.cursor[t] = pa;
        const unsigned nf = e / ie, rem = e % ie;
        for (unsigned i = 0u; i < nf; ++i) S.item_desc[pb + i] = make_uint4((unsigned)t, pa + i * ie, ie, 1u);
        if (rem) S.item_desc[atomicAdd(&s_roff[rem], 1u)] = make_uint4((unsigned)t, pa + nf * ie, rem, 1u);
        pa += e;
        pb += nf;
        S.tile_ent[t] = 0u;
        S.tile_rec[t] = 0u;
    }
    if (threadIdx.x == blockDim.x - 1) {
        const unsigned recs = s_r[threadIdx.x];
        SweepCtl* c = S.ctl;
        S.ent_off[n] = s_a[threadIdx.x];
        c->n_items = s_roff[0];
        c->item_next = 0u;
        const bool emitted_all = c->emitted >= S.n_packets;
        if (emitted_all && recs != 0u && recs <= S.drain_below) {
            // few records left and nothing more to emit: the per-lane finish
            // takes buffer b's entries as they are, and no sweep walks them
            c->drain = 1u;
            c->drain_buf = (unsigned)b;
            c->drain_next = 0u;
            c->drain_recs = recs;
            c->n_items = 0u;
            c->done = 1u;
            return;
        }
        c->visits += recs;
        if (recs) c->sweeps += 1u;
        c->done = (recs == 0u && emitted_all) ? 1u : 0u;
        c->rec_alloc[b ^ 1] = 0u;
        c->n_ent[b ^ 1] = 0u;
    }
}

// Entries of buffer b grouped by tile.  A block takes kGroupStep entries at
// a time, ranks them per tile in LDS, reserves each tile's range with one
// atomic on the tile's cursor, and writes every entry at its range plus its
// rank (the entries of a hot tile then cost one global atomic per block step,
// not one each).  Grids of more than kGroupTiles tiles rank with one global
// atomic per entry.
constexpr int kGroupPer = 8;
constexpr int kGroupStep = kGroupPer * 256;
constexpr int kGroupTiles = 4096;

__global__ void __launch_bounds__(256) k_sweep_group(SweepParams S, int b) {
    __shared__ unsigned s_rank[kGroupTiles];
    if (S.ctl->drain) return;
    const unsigned n = S.ctl->n_ent[b] < S.max_ent ? S.ctl->n_ent[b] : S.max_ent;
    if (S.ntiles > kGroupTiles) {
        for (unsigned e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
            const uint2 en = S.ent[b][e];
            if (en.y == 0u) continue;  // a slot a wave held but did not use
            S.sent[atomicAdd(S.cursor + S.ent_tile[b][e], 1u)] = en;
        }
        return;
    }
    for (unsigned c0 = blockIdx.x * (unsigned)kGroupStep; c0 < n; c0 += gridDim.x * (unsigned)kGroupStep) {
        for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x) s_rank[t] = 0u;
        __syncthreads();
        unsigned tl[kGroupPer], rk[kGroupPer];
        uint2 en[kGroupPer];
#pragma unroll
        for (int j = 0; j < kGroupPer; ++j) {
            const unsigned e = c0 + (unsigned)(j * 256) + threadIdx.x;
            tl[j] = kNone;
            if (e < n) {
                en[j] = S.ent[b][e];
                if (en[j].y != 0u) {
                    tl[j] = S.ent_tile[b][e];
                    rk[j] = atomicAdd(&s_rank[tl[j]], 1u);
                }
            }
        }
        __syncthreads();
        for (int t = threadIdx.x; t < S.ntiles; t += blockDim.x)
            if (s_rank[t]) s_rank[t] = atomicAdd(S.cursor + t, s_rank[t]);  // count -> range start
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kGroupPer; ++j)
            if (tl[j] != kNone) S.sent[s_rank[tl[j]] + rk[j]] = en[j];
        __syncthreads();
    }
}

// ---- the sweep ------------------------------------------------------------------
// The tile's density into LDS and its tally cleared: 16-byte loads, eight in
// flight per thread, when the tile lies inside the grid and its rows are
// aligned; otherwise cell by cell.
template <typename R>
__device__ __forceinline__ void load_tile(const TransportParams<R>& P, int o0, int o1, int o2, int txy,
                                          int tz, R* rho_t, double* acc_t, double* acc2_t) {
    constexpr int VW = 16 / (int)sizeof(R);
    using V = typename std::conditional<sizeof(R) == 4, float4, double2>::type;
    const int tcells = txy * txy * tz;
    const bool vec = o0 + txy <= P.n[0] && o1 + txy <= P.n[1] && o2 + tz <= P.n[2] && P.n[0] % VW == 0 &&
                     txy % VW == 0;
    if (vec) {
        const int nv = tcells / VW, per_row = txy / VW;
        const int bd = (int)blockDim.x;
        auto src = [&](int q) {
            const int row = q / per_row, part = q - row * per_row;
            const int ly = row % txy, lz = row / txy;
            return reinterpret_cast<const V*>(
                P.rho + ((o0 + part * VW) + (int64_t)P.n[0] * ((o1 + ly) + (int64_t)P.n[1] * (o2 + lz))));
        };
        // eight loads in flight per thread (a guarded load of a vector past the
        // tile's end reads vector 0 and is not stored)
        V* r = reinterpret_cast<V*>(rho_t);
        for (int q0 = threadIdx.x; q0 < nv; q0 += 8 * bd) {
            const int q1 = q0 + bd, q2 = q0 + 2 * bd, q3 = q0 + 3 * bd, q4 = q0 + 4 * bd;
            const int q5 = q0 + 5 * bd, q6 = q0 + 6 * bd, q7 = q0 + 7 * bd;
            const V v0 = *src(q0);
            const V v1 = *src(q1 < nv ? q1 : 0), v2 = *src(q2 < nv ? q2 : 0), v3 = *src(q3 < nv ? q3 : 0);
            const V v4 = *src(q4 < nv ? q4 : 0), v5 = *src(q5 < nv ? q5 : 0), v6 = *src(q6 < nv ? q6 : 0);
            const V v7 = *src(q7 < nv ? q7 : 0);
            r[q0] = v0;
            if (q1 < nv) r[q1] = v1;
            if (q2 < nv) r[q2] = v2;
            if (q3 < nv) r[q3] = v3;
            if (q4 < nv) r[q4] = v4;
            if (q5 < nv) r[q5] = v5;
            if (q6 < nv) r[q6] = v6;
            if (q7 < nv) r[q7] = v7;
        }
    } else {
        for (int i = threadIdx.x; i < tcells; i += blockDim.x) {
            const int lx = i % txy, ly = (i / txy) % txy, lz = i / (txy * txy);
            const int gx = o0 + lx, gy = o1 + ly, gz = o2 + lz;
            R r = (R)0;
            if (gx < P.n[0] && gy < P.n[1] && gz < P.n[2])
                r = P.rho[gx + (int64_t)P.n[0] * (gy + (int64_t)P.n[1] * gz)];
            rho_t[i] = r;
        }
    }
    // the FP64 tally (and sum of squares) cleared, 16 bytes at a time
    const int nd = (acc2_t ? 2 : 1) * tcells;  // doubles; the two arrays are adjacent
    const double2 z2 = make_double2(0.0, 0.0);
    for (int i = threadIdx.x; i < nd / 2; i += blockDim.x) reinterpret_cast<double2*>(acc_t)[i] = z2;
    if ((nd & 1) && threadIdx.x == 0) acc_t[nd - 1] = 0.0;
}

// The tile's LDS partial sums into the FP64 tally (cells of this tile only).
template <typename R>
__device__ __forceinline__ void flush_tile(const TransportParams<R>& P, int o0, int o1, int o2, int txy,
                                           int tcells, const double* acc_t, const double* acc2_t) {
    for (int i = threadIdx.x; i < tcells; i += blockDim.x) {
        const double a = acc_t[i];
        const double a2 = acc2_t ? acc2_t[i] : 0.0;
        if (a != 0.0 || a2 != 0.0) {
            const int lx = i % txy, ly = (i / txy) % txy, lz = i / (txy * txy);
            const int64_t j = (o0 + lx) + (int64_t)P.n[0] * ((o1 + ly) + (int64_t)P.n[1] * (o2 + lz));
            if (a != 0.0) unsafeAtomicAdd(P.acc + j, a);
            if (a2 != 0.0) unsafeAtomicAdd(P.acc2 + j, a2);
        }
    }
}

// Wave 0 of a group claims a work item and stages its descriptor (tile, first
// entry, entry count, 1) and its entries in LDS slot `slot`; no item left
// gives a descriptor with w = 0.
__device__ __forceinline__ void stage_item(const SweepParams& S, unsigned n_items, uint4* s_desc,
                                           uint2* s_ent, int slot, int lane) {
    unsigned item = 0u;
    if (lane == 0) item = atomicAdd(&S.ctl->item_next, 1u);
    item = (unsigned)__shfl((int)item, 0);
    if (item >= n_items) {
        if (lane == 0) s_desc[slot] = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    const uint4 d = S.item_desc[item];
    for (unsigned i = (unsigned)lane; i < d.z; i += 64u) s_ent[i] = S.sent[d.y + i];
    if (lane == 0) s_desc[slot] = d;
}

// One sweep: reads the records of buffer b (entries grouped in S.sent),
// writes the records that stay in flight into buffer b^1.  Persistent
// workgroups, one per compute unit (the tile takes most of its LDS); in FP32
// of up to 768 threads in the lean kernel (three waves per SIMD fit its
// registers) and 512 in the full one; the FP64 walk keeps 256 threads.
template <typename R, bool NOISE, bool FULL>
__global__ void __launch_bounds__(sizeof(R) == 4 ? (FULL ? 512 : 768) : 256) k_sweep(TransportParams<R> P, SweepParams S,
                                                                      int b) {
    constexpr int K = 4;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ unsigned s_enext, s_eend, s_stager;
    __shared__ uint4 s_desc[2];                  // the current and the next work item
    __shared__ uint2 s_ents[2][kMaxItemEnt];     // and their entries
    __shared__ unsigned s_tc[14];          // records, entries registered per destination slot
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    if (S.ctl->drain) return;  // the tail went to the per-lane finish
    const int bo = b ^ 1;  // the buffer this sweep writes
    const int txy = S.txy;
    const int tcells = txy * txy * S.tz;
    // LDS: Sum w^2 (FP64, when kept), density, tally, the bins' chi, kappa,
    // albedo and g, the luminosity CDF and the coarse CDF indices (the host
    // sizes the tile so that all of it fits): everything the walk and the
    // events read per packet, so that no global load feeds the walk
    double* acc_t = reinterpret_cast<double*>(smem_raw);
    double* acc2_t = NOISE ? acc_t + tcells : nullptr;
    R* rho_t = reinterpret_cast<R*>(acc_t + (NOISE ? 2 : 1) * tcells);
    R* chi_t = rho_t + tcells;
    R* kap_t = chi_t + P.nnu;
    R* alb_t = kap_t + P.nnu;
    R* g_t = alb_t + P.nnu;
    R* sm_tab = g_t + P.nnu;
    for (int i = threadIdx.x; i < P.nnu; i += blockDim.x) {
        chi_t[i] = P.chi[i];
        kap_t[i] = P.kap[i];
        alb_t[i] = P.alb[i];
        g_t[i] = P.g[i];
    }
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    const int ne = kRows * P.ngroup, ns = P.nsrc * P.ngroup;
    for (int i = threadIdx.x; i < P.nsrc; i += blockDim.x) sm_tab[i] = P.lcdf[i];
    for (int i = threadIdx.x; i < ne; i += blockDim.x) sm_tab[P.nsrc + i] = P.ecoarse[i];
    for (int i = threadIdx.x; i < ns; i += blockDim.x) sm_tab[P.nsrc + ne + i] = P.scoarse[i];
    const Tables<R> tb{sm_tab, sm_tab + P.nsrc, sm_tab + P.nsrc + ne, chi_t, kap_t, alb_t, g_t};
    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    const int lane = __lane_id();
    const int service = S.service;
    const uint4* in = S.recs[b];
    Stream<R> rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.n = 0;
    rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    const unsigned n_items = S.ctl->n_items;
    int tile = -1;  // the tile held in LDS (block-uniform)
    int o0 = 0, o1 = 0, o2 = 0;
    WaveOut wo;
    wave_out_init(wo);
    if (threadIdx.x < 14) s_tc[threadIdx.x] = 0u;

    // Work items are claimed one ahead: the first wave to finish an item (it
    // would wait at the barrier anyway) claims the next one and stages its
    // descriptor and entries in the other LDS slot, so that an item boundary
    // costs only the barriers (and the tile change, if any).
    if (threadIdx.x < 64) stage_item(S, n_items, s_desc, s_ents[0], 0, lane);
    if (threadIdx.x == 0) s_stager = 0u;
    int cur = 0;
    for (;;) {
        __syncthreads();
        const uint4 d = s_desc[cur];
        if (d.w == 0u) break;
        const int ti = (int)d.x;
        if (ti != tile) {
            // an item of the tile already in LDS keeps it; otherwise the tile
            // in LDS goes out before the item's tile comes in
            if (tile >= 0) {
                chunks_close(S, bo, tile, wo, s_tc, lane);
                __syncthreads();
                flush_tile_counts(S, tile, s_tc);
                flush_tile(P, o0, o1, o2, txy, tcells, acc_t, acc2_t);
                __syncthreads();
            }
            tile = ti;
            const int tzi = tile / (S.ntx * S.nty);
            const int trem = tile - tzi * S.ntx * S.nty;
            const int tyi = trem / S.ntx, txi = trem - tyi * S.ntx;
            o0 = txi * txy;
            o1 = tyi * txy;
            o2 = tzi * S.tz;
            load_tile(P, o0, o1, o2, txy, S.tz, rho_t, acc_t, acc2_t);
        }
        if (threadIdx.x == 0) {
            s_enext = 0u;
            s_eend = d.z;
            s_stager = 0u;
        }
        __syncthreads();

        // the wave's current entry: records [eb + ep, eb + ec) not yet handed out
        unsigned eb = 0u, ec = 0u, ep = 0u;
        bool drained = false;  // the item has no entry left for this wave (wave-uniform)
        Packet<R> s;
        s.st = ST_EMPTY;
        Raw<R> nx;             // the record this lane walks next
        bool hn = false;       // nx holds one
        int jl = 0;            // the packet's cell in LDS
        R rho = (R)0;          // and its density
        int visit = 0;
        for (;;) {
            // events, escapes, exits
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
                    interact<R, TileDeposit<R>, FULL, true>(s, rs, P, tb, cnt, e_killed,
                                                            TileDeposit<R>{acc_t, acc2_t, o0, o1, o2, txy});
                }
            }
            if (s.st == ST_ESC) escape<R, FULL>(s, P, cnt, e_escaped);
            write_exits(S, bo, tile, o0, o1, o2, s, rs, wo, s_tc, lane);
            // free lanes take their next record
            if (s.st == ST_EMPTY && hn) {
                unpack_rec(s, rs, P, nx, tb.chi, tb.kap);
                hn = false;
                if (s.st != ST_EMPTY) {
                    // a record always lies in the tile it was registered for;
                    // anything else is dropped and reported
                    if ((unsigned)(s.c0 - o0) >= (unsigned)txy || (unsigned)(s.c1 - o1) >= (unsigned)txy ||
                        (unsigned)(s.c2 - o2) >= (unsigned)S.tz || !in_grid(P, s.c0, s.c1, s.c2)) {
                        atomicOr(&S.ctl->overflow, 2u);
                        s.st = ST_EMPTY;
                    } else {
                        jl = tile_index(s.c0, s.c1, s.c2, o0, o1, o2, txy);
                        rho = rho_t[jl];
                        visit = 0;
                        if (s.st == ST_EVENT)
                            s.rowp = P.rowpos[grid_index(P, s.c0, s.c1, s.c2)];
                    }
                }
            }
            // and lanes without a next record claim one from the wave's entry
            for (;;) {
                const unsigned long long need = __ballot(!hn);
                if (need == 0ull || drained) break;
                if (ep == ec) {
                    unsigned e = 0u;
                    if (lane == 0) e = atomicAdd(&s_enext, 1u);
                    e = (unsigned)__shfl((int)e, 0);
                    if (e >= s_eend) {
                        drained = true;
                        break;
                    }
                    const uint2 en = s_ents[cur][e];
                    eb = (unsigned)__builtin_amdgcn_readfirstlane(en.x);
                    ec = (unsigned)__builtin_amdgcn_readfirstlane(en.y);
                    ep = 0u;
                    continue;
                }
                const unsigned avail = ec - ep;
                const unsigned rank = (unsigned)__popcll(need & __lanemask_lt());
                if (!hn && rank < avail) {
                    load_raw(S, in, eb + ep + rank, nx);
                    hn = true;
                }
                const unsigned n = (unsigned)__popcll(need);
                ep += n < avail ? n : avail;
            }
            if (__ballot(s.st != ST_EMPTY || hn) == 0ull && drained) {
                unsigned first = 1u;
                if (lane == 0) first = atomicAdd(&s_stager, 1u);
                if (__shfl((int)first, 0) == 0) stage_item(S, n_items, s_desc, s_ents[cur ^ 1], cur ^ 1, lane);
                break;
            }
            // walk until `service` lanes wait (or none walks)
            for (;;) {
                if (s.st == ST_WALK)
                    walk_tile<R, K, NOISE>(s, P, o0, o1, o2, txy, S.tz, rho_t, acc_t, acc2_t, cnt, jl, rho);
                if (__ballot(s.st == ST_WALK) == 0ull) break;
                const bool wait = s.st != ST_WALK && (s.st != ST_EMPTY || hn || !drained);
                if (__popcll(__ballot(wait)) >= service) break;
            }
        }
        cur ^= 1;
    }
    if (tile >= 0) {
        chunks_close(S, bo, tile, wo, s_tc, lane);
        __syncthreads();
        flush_tile_counts(S, tile, s_tc);
        flush_tile(P, o0, o1, o2, txy, tcells, acc_t, acc2_t);
    }
    wave_out_release(S, bo, wo, lane);
    flush_block_counters(P, cnt, e_escaped, e_killed, s_cnt, s_energy);
}

// The tail of a pass.  Once every packet is emitted and at most drain_below
// records remain, each further sweep would cost a kernel's start and end for
// a few records of long-lived packets; instead the records of buffer b are
// finished by the per-lane walk over the whole grid (global density and FP64
// tally, the arithmetic of the tiled walk segment by segment), as in the
// per-lane transport.  A wave takes one entry at a time and finishes its
// records 64 at a time.
template <typename R>
__global__ void __launch_bounds__(256) k_sweep_drain(TransportParams<R> P, SweepParams S, int b) {
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    __syncthreads();
    const Tables<R> tb = global_tables(P);
    uint32_t cnt[C_COUNT];
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) cnt[c] = 0u;
    double e_escaped = 0.0, e_killed = 0.0;
    const int lane = __lane_id();
    const unsigned n = S.ctl->n_ent[b] < S.max_ent ? S.ctl->n_ent[b] : S.max_ent;
    for (;;) {
        unsigned e = 0u;
        if (lane == 0) e = atomicAdd(&S.ctl->drain_next, 1u);
        e = __shfl(e, 0);
        if (e >= n) break;
        // (first record, count); count 0: an unused slot; a chunk holds at
        // most 64 records, an emission run up to a block's step
        const uint2 en = S.ent[b][e];
        for (unsigned o = 0u; o < en.y; o += 64u) {
            Packet<R> s;
            s.st = ST_EMPTY;
            Stream<R> rs;
            rs.k0 = P.key0;
            rs.k1 = P.key1;
            rs.n = 0;
            rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
            if (o + (unsigned)lane < en.y) {
                Raw<R> r;
                load_raw<R>(S, S.recs[b], en.x + o + (unsigned)lane, r);
                unpack_rec(s, rs, P, r, tb.chi, tb.kap);
            }
            while (s.st == ST_WALK || s.st == ST_EVENT || s.st == ST_ESC) {
                if (s.st == ST_WALK) walk<R, 4, 0>(s, P, P.acc, cnt);
                if (s.st == ST_EVENT) interact(s, rs, P, tb, cnt, e_killed, global_deposit<0>(P, P.acc));
                if (s.st == ST_ESC) escape(s, P, cnt, e_escaped);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) atomicAdd(&s_cnt[c], (unsigned long long)cnt[c]);
    atomicAdd(&s_energy[0], e_escaped);
    atomicAdd(&s_energy[1], e_killed);
    __syncthreads();
    if (threadIdx.x < C_COUNT) atomicAdd(P.counters + threadIdx.x, s_cnt[threadIdx.x]);
    if (threadIdx.x < 2) unsafeAtomicAdd(P.energies + threadIdx.x, s_energy[threadIdx.x]);
}

template <typename R>
hipError_t launch_sweep_drain(const TransportParams<R>& P, const SweepParams& S, int b, int blocks,
                              hipStream_t st) {
    hipLaunchKernelGGL(k_sweep_drain<R>, dim3(blocks), dim3(256), 0, st, P, S, b);
    return hipGetLastError();
}
template hipError_t launch_sweep_drain<float>(const TransportParams<float>&, const SweepParams&, int, int,
                                              hipStream_t);
template hipError_t launch_sweep_drain<double>(const TransportParams<double>&, const SweepParams&, int, int,
                                               hipStream_t);

__global__ void k_fill_u32(unsigned* p, int n, unsigned v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
size_t sweep_record_bytes(int fp32) { return 16u * (fp32 ? Rec<float>::NQ : Rec<double>::NQ); }

template <typename R> using SweepFn = void (*)(TransportParams<R>, SweepParams, int);

template <typename R> SweepFn<R> pick_sweep(bool noise, bool full) {
    if (noise) return full ? k_sweep<R, true, true> : k_sweep<R, true, false>;
    return full ? k_sweep<R, false, true> : k_sweep<R, false, false>;
}

// One step of the sweeps; the events (may be null) bracket the sweep kernel,
// the pass's dominant kernel.
template <typename R>
hipError_t launch_sweep_step(const TransportParams<R>& P, const SweepParams& S, int b, bool full,
                             int emit_blocks, int group_blocks, int blocks, int threads, size_t lds,
                             hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
    hipLaunchKernelGGL(k_refill_plan, dim3(1), dim3(1024), 0, st, S, b);
    if (full) hipLaunchKernelGGL((k_sweep_emit<R, true>), dim3(emit_blocks), dim3(kEmitThreads), 0, st, P, S, b);
    else hipLaunchKernelGGL((k_sweep_emit<R, false>), dim3(emit_blocks), dim3(kEmitThreads), 0, st, P, S, b);
    hipLaunchKernelGGL(k_sweep_scan, dim3(1), dim3(1024), 0, st, S, b);
    hipLaunchKernelGGL(k_sweep_group, dim3(group_blocks), dim3(256), 0, st, S, b);
    if (ev0) {
        const hipError_t e = hipEventRecord(ev0, st);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(pick_sweep<R>(P.acc2 != nullptr, full), dim3(blocks), dim3(threads), lds, st, P, S, b);
    if (ev1) {
        const hipError_t e = hipEventRecord(ev1, st);
        if (e != hipSuccess) return e;
    }
    return hipGetLastError();
}

template <typename R> hipError_t sweep_prepare(bool noise, bool full, size_t lds) {
    if (lds <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(pick_sweep<R>(noise, full)),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename R> int sweep_max_blocks_per_cu(bool noise, bool full, int threads, size_t lds) {
    int nb = 0;
    if (sweep_prepare<R>(noise, full, lds) != hipSuccess) return 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_sweep<R>(noise, full), threads, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

int sweep_emit_step() { return kEmitStep; }

hipError_t launch_fill_u32(unsigned* p, int n, unsigned v, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024), dim3(256), 0,
                       st, p, n, v);
    return hipGetLastError();
}

template hipError_t launch_sweep_step<float>(const TransportParams<float>&, const SweepParams&, int, bool,
                                             int, int, int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t launch_sweep_step<double>(const TransportParams<double>&, const SweepParams&, int, bool,
                                              int, int, int, int, size_t, hipStream_t, hipEvent_t, hipEvent_t);
template hipError_t sweep_prepare<float>(bool, bool, size_t);
template hipError_t sweep_prepare<double>(bool, bool, size_t);
template int sweep_max_blocks_per_cu<float>(bool, bool, int, size_t);
template int sweep_max_blocks_per_cu<double>(bool, bool, int, size_t);

}  // namespace mcrt
