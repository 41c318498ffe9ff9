// mcrt_transport.hip -- photon-packet transport for gfx950 (Robitaille 2011,
// Sec. 2.2 propagation, Sec. 2.3 Eq. 2 Lucy estimator, Sec. 2.6.1 binning).
//
// One persistent launch processes a whole pass.  Every lane of a wave64 holds
// one packet in registers.  Lanes that have finished a packet take new packet
// ids from a chunk that the wave draws from the global pool counter (pool
// refill, one global atomic per 64 packets).  Between events a lane walks the
// grid in batches of K segments: it first steps the ray K walls ahead (pure
// arithmetic, Amanatides-Woo style: per axis the ray distance of the next wall
// and the distance between walls), then issues the K density gathers at once,
// then consumes the segments in order, adding weight*l*kappa to each dust
// cell's FP64 absorption tally with a hardware FP64 atomic, until the sampled
// optical depth is used up.  K gathers in flight per lane instead of one hide
// the memory latency that otherwise bounds the walk.
//
// A wave keeps walking until `defer_lanes` of its lanes wait for an event and
// then handles all waiting lanes of one event type together (event-type
// compaction by ballot).  Frequency sampling uses a two-level search: a
// coarse index of every 16th CDF entry staged in LDS, then one 64-byte group
// read from global memory.
//
// The grid arrays may be stored in bricks of 4x4x4 cells so that the few
// cells a ray crosses inside a brick share cache lines.
//
// The same template serves the FP64 path (same random stream and decisions as
// the CPU oracle) and the FP32 transport form.
#include <math.h>

#include "mcrt_internal.h"
#include "mcrt_packet.h"

namespace mcrt {

template <typename R, int K, int BRICK>
__global__ void __launch_bounds__(256) k_transport(TransportParams<R> P) {
    extern __shared__ unsigned char smem_raw[];
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
    Tables<R> tb = global_tables(P);
    if (P.lds_tables) {
        R* sm = reinterpret_cast<R*>(smem_raw);
        const int ne = kRows * P.ngroup, ns = P.nsrc * P.ngroup;
        for (int i = threadIdx.x; i < P.nsrc; i += blockDim.x) sm[i] = P.lcdf[i];
        for (int i = threadIdx.x; i < ne; i += blockDim.x) sm[P.nsrc + i] = P.ecoarse[i];
        for (int i = threadIdx.x; i < ns; i += blockDim.x) sm[P.nsrc + ne + i] = P.scoarse[i];
        tb.lcdf = sm;
        tb.ecoarse = sm + P.nsrc;
        tb.scoarse = sm + P.nsrc + ne;
    } else {
        tb.lcdf = P.lcdf;
        tb.ecoarse = P.ecoarse;
        tb.scoarse = P.scoarse;
    }
    __syncthreads();

    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    Packet<R> s;
    s.st = ST_EMPTY;
    s.id = 0;
    Stream<R> rs;
    rs.k0 = P.key0;
    rs.k1 = P.key1;
    rs.n = 0;
    rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    const int lane = __lane_id();
    const int defer = P.defer_lanes;
    // absorption tally of this block: with per-XCD copies, the copy of the XCD
    // the block runs on (hardware XCC id), so that the FP64 atomics of different
    // XCDs never meet on a cache line
    double* acc = P.acc;
    if (P.acc_stride) {
        unsigned xcc;
        asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
        acc += (size_t)(xcc & 7u) * P.acc_stride;
    }
    // packet ids held by this wave: [wbase, wend), the same value in every lane
    uint64_t wbase = 0, wend = 0;

    for (;;) {
        // pool refill: empty lanes take ids from the wave's chunk, which is
        // topped up from the global pool with one atomic per kPoolChunk ids
        const unsigned long long need = __ballot(s.st == ST_EMPTY);
        if (need) {
            const int nneed = __popcll(need);
            const int rank = __popcll(need & __lanemask_lt());
            const int avail = (int)(wend - wbase);
            const int take = nneed < avail ? nneed : avail;
            uint64_t my = wbase + (uint64_t)rank;
            wbase += (uint64_t)take;
            if (nneed > take) {
                const int leader = __ffsll((long long)need) - 1;
                unsigned long long g = 0;
                if (lane == leader) g = atomicAdd(P.pool, (unsigned long long)kPoolChunk);
                g = shfl_u64(g, leader);
                if (rank >= take) my = g + (uint64_t)(rank - take);
                wbase = g + (uint64_t)(nneed - take);
                wend = g + kPoolChunk;
            }
            if (s.st == ST_EMPTY) {
                if (my < P.n_packets) emit(s, rs, P, tb, my, cnt, e_killed, global_deposit<BRICK>(P, acc));
                else s.st = ST_DONE;
            }
        }
        if (__ballot(s.st != ST_DONE) == 0ull) break;
        // walk until enough lanes wait for an event (or none walks)
        for (;;) {
            if (s.st == ST_WALK) walk<R, K, BRICK>(s, P, acc, cnt);
            if (__ballot(s.st == ST_WALK) == 0ull) break;
            if (__popcll(__ballot(s.st == ST_EVENT || s.st == ST_ESC)) >= defer) break;
        }
        if (s.st == ST_EVENT) interact(s, rs, P, tb, cnt, e_killed, global_deposit<BRICK>(P, acc));
        if (s.st == ST_ESC) escape(s, P, cnt, e_escaped);
    }

#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) atomicAdd(&s_cnt[c], (unsigned long long)cnt[c]);
    atomicAdd(&s_energy[0], e_escaped);
    atomicAdd(&s_energy[1], e_killed);
    __syncthreads();
    if (threadIdx.x < C_COUNT) atomicAdd(P.counters + threadIdx.x, s_cnt[threadIdx.x]);
    if (threadIdx.x < 2) unsafeAtomicAdd(P.energies + threadIdx.x, s_energy[threadIdx.x]);
}

template <typename R> using KernelFn = void (*)(TransportParams<R>);

template <typename R> KernelFn<R> pick_kernel(int K, int brick) {
    if (brick) {
        switch (K) {
            case 1: return k_transport<R, 1, 1>;
            case 2: return k_transport<R, 2, 1>;
            case 8: return k_transport<R, 8, 1>;
            default: return k_transport<R, 4, 1>;
        }
    }
    switch (K) {
        case 1: return k_transport<R, 1, 0>;
        case 2: return k_transport<R, 2, 0>;
        case 8: return k_transport<R, 8, 0>;
        default: return k_transport<R, 4, 0>;
    }
}

template <typename R>
size_t transport_lds_bytes(const TransportParams<R>& P) {
    return P.lds_tables ? (size_t)(P.nsrc + (kRows + P.nsrc) * P.ngroup) * sizeof(R) : 0;
}

template <typename R>
hipError_t launch_transport(const TransportParams<R>& P, int K, int brick, int blocks, int threads,
                            hipStream_t st) {
    hipLaunchKernelGGL(pick_kernel<R>(K, brick), dim3(blocks), dim3(threads),
                       transport_lds_bytes(P), st, P);
    return hipGetLastError();
}

template <typename R> int transport_max_blocks_per_cu(int K, int brick, int threads, size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_kernel<R>(K, brick), threads, lds) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template hipError_t launch_transport<double>(const TransportParams<double>&, int, int, int, int,
                                             hipStream_t);
template hipError_t launch_transport<float>(const TransportParams<float>&, int, int, int, int,
                                            hipStream_t);
template int transport_max_blocks_per_cu<double>(int, int, int, size_t);
template int transport_max_blocks_per_cu<float>(int, int, int, size_t);
template size_t transport_lds_bytes<double>(const TransportParams<double>&);
template size_t transport_lds_bytes<float>(const TransportParams<float>&);

// ---------------------------------------------------------------------------
// Batched transport: many independent models in one persistent launch.
// The packets of all models form one pool of 64-id chunks; chunk c belongs to
// the model m with chunk_start[m] <= c < chunk_start[m+1].  Each lane reads the
// launch parameters of its packet's model from device memory, so the lanes of
// a wave may work on different models.  Each model keeps its own random
// streams (its seed and iteration), tallies and counters: a model's results
// equal those of its own single-model launch up to summation order.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void flush_counters(unsigned long long* counters, double* energies,
                                               uint32_t* cnt, double& e_esc, double& e_kill) {
#pragma unroll
    for (int c = 0; c < C_COUNT; ++c) {
        if (cnt[c]) atomicAdd(counters + c, (unsigned long long)cnt[c]);
        cnt[c] = 0;
    }
    if (e_esc != 0.0) unsafeAtomicAdd(energies + 0, e_esc);
    if (e_kill != 0.0) unsafeAtomicAdd(energies + 1, e_kill);
    e_esc = 0.0;
    e_kill = 0.0;
}

template <typename R, int K, int BRICK>
__global__ void __launch_bounds__(256)
k_transport_batch(const TransportParams<R>* __restrict__ Ps,
                  const unsigned long long* __restrict__ chunk_start, int n_models,
                  unsigned long long* pool, const uint32_t* __restrict__ keys) {
    const unsigned long long total = chunk_start[n_models];
    uint32_t cnt[C_COUNT] = {0, 0, 0, 0, 0, 0};
    double e_escaped = 0.0, e_killed = 0.0;
    unsigned xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    Packet<R> s;
    s.st = ST_EMPTY;
    s.id = 0;
    Stream<R> rs;
    rs.n = 0;
    rs.k0 = rs.k1 = rs.p0 = rs.p1 = rs.s0 = rs.s1 = 0;
    const int lane = __lane_id();
    int lm = -1;     // model of the lane's packet (and of its counters)
    // the wave's chunk: model wm, ids [wbase, wend) -- the same in every lane
    int wm = 0;
    uint64_t wbase = 0, wend = 0;
    bool drained = false;

    for (;;) {
        unsigned long long need = __ballot(s.st == ST_EMPTY);
        while (need && !drained) {
            if (wbase >= wend) {
                unsigned long long c = 0;
                const int leader = __ffsll((long long)need) - 1;
                if (lane == leader) c = atomicAdd(pool, 1ull);
                c = shfl_u64(c, leader);
                if (c >= total) {
                    drained = true;
                    break;
                }
                int lo = 0, hi = n_models - 1;  // last m with chunk_start[m] <= c
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (chunk_start[mid] <= c) lo = mid;
                    else hi = mid - 1;
                }
                wm = lo;
                wbase = (c - chunk_start[wm]) * (uint64_t)kPoolChunk;
                const uint64_t np = Ps[wm].n_packets;
                wend = wbase + kPoolChunk < np ? wbase + kPoolChunk : np;
                continue;
            }
            const int avail = (int)(wend - wbase);
            const int nneed = __popcll(need);
            const int take = nneed < avail ? nneed : avail;
            const int rank = __popcll(need & __lanemask_lt());
            if (s.st == ST_EMPTY && rank < take) {
                if (lm != wm) {
                    if (lm >= 0)
                        flush_counters(Ps[lm].counters, Ps[lm].energies, cnt, e_escaped, e_killed);
                    lm = wm;
                }
                const TransportParams<R>& P = Ps[lm];
                const Tables<R> tb = global_tables(P);
                rs.k0 = P.key0;
                rs.k1 = keys[lm];
                emit(s, rs, P, tb, wbase + (uint64_t)rank, cnt, e_killed, global_deposit<BRICK>(P, P.acc));
            }
            wbase += (uint64_t)take;
            need = __ballot(s.st == ST_EMPTY);
        }
        if (drained && s.st == ST_EMPTY) s.st = ST_DONE;
        if (__ballot(s.st != ST_DONE) == 0ull) break;
        const int mm = lm < 0 ? 0 : lm;
        const TransportParams<R>& P = Ps[mm];
        double* acc = P.acc + (P.acc_stride ? (size_t)(xcc & 7u) * P.acc_stride : (size_t)0);
        const int defer = Ps[0].defer_lanes;  // the same for every lane of the wave
        WalkGrid<R> wg;
        wg.n[0] = P.n[0];
        wg.n[1] = P.n[1];
        wg.n[2] = P.n[2];
        wg.bx = P.bx;
        wg.bxy = P.bxy;
        wg.rho = P.rho;
        wg.acc2 = P.acc2;
        for (;;) {
            if (s.st == ST_WALK) walk<R, K, BRICK>(s, wg, acc, cnt);
            if (__ballot(s.st == ST_WALK) == 0ull) break;
            if (__popcll(__ballot(s.st == ST_EVENT || s.st == ST_ESC)) >= defer) break;
        }
        const Tables<R> tb = global_tables(P);
        if (s.st == ST_EVENT) interact(s, rs, P, tb, cnt, e_killed, global_deposit<BRICK>(P, acc));
        if (s.st == ST_ESC) escape(s, P, cnt, e_escaped);
    }
    if (lm >= 0) flush_counters(Ps[lm].counters, Ps[lm].energies, cnt, e_escaped, e_killed);
}

template <typename R> using BatchFn = void (*)(const TransportParams<R>*, const unsigned long long*,
                                               int, unsigned long long*, const uint32_t*);

template <typename R> BatchFn<R> pick_batch_kernel(int K, int brick) {
    if (brick) {
        switch (K) {
            case 2: return k_transport_batch<R, 2, 1>;
            case 8: return k_transport_batch<R, 8, 1>;
            default: return k_transport_batch<R, 4, 1>;
        }
    }
    switch (K) {
        case 2: return k_transport_batch<R, 2, 0>;
        case 8: return k_transport_batch<R, 8, 0>;
        default: return k_transport_batch<R, 4, 0>;
    }
}

template <typename R>
hipError_t launch_transport_batch(const TransportParams<R>* Ps, const unsigned long long* chunk_start,
                                  int n_models, unsigned long long* pool, const uint32_t* keys,
                                  int K, int brick, int blocks, int threads, hipStream_t st) {
    hipLaunchKernelGGL(pick_batch_kernel<R>(K, brick), dim3(blocks), dim3(threads), 0, st, Ps,
                       chunk_start, n_models, pool, keys);
    return hipGetLastError();
}

template <typename R> int batch_max_blocks_per_cu(int K, int brick, int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, pick_batch_kernel<R>(K, brick), threads,
                                                     0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template hipError_t launch_transport_batch<double>(const TransportParams<double>*,
                                                   const unsigned long long*, int,
                                                   unsigned long long*, const uint32_t*, int, int,
                                                   int, int, hipStream_t);
template hipError_t launch_transport_batch<float>(const TransportParams<float>*,
                                                  const unsigned long long*, int,
                                                  unsigned long long*, const uint32_t*, int, int,
                                                  int, int, hipStream_t);
template int batch_max_blocks_per_cu<double>(int, int, int);
template int batch_max_blocks_per_cu<float>(int, int, int);

// ---------------------------------------------------------------------------
// The direction update of a scattering (Sec. 2.2, Henyey-Greenstein angle mu
// and azimuth phi about the incoming direction), n directions at a time, in
// the transport precision R: the device function every transport kernel uses.
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_rotate(const double* __restrict__ d, const double* __restrict__ mu,
                         const double* __restrict__ phi, double* __restrict__ out, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R d0 = (R)d[3 * i], d1 = (R)d[3 * i + 1], d2 = (R)d[3 * i + 2];
    rotate_dir<R>(d0, d1, d2, (R)mu[i], (R)phi[i]);
    out[3 * i] = (double)d0;
    out[3 * i + 1] = (double)d1;
    out[3 * i + 2] = (double)d2;
}

hipError_t launch_rotate(int fp32, const double* d, const double* mu, const double* phi, double* out,
                         int n, hipStream_t st) {
    const int blocks = (n + 255) / 256;
    if (fp32) hipLaunchKernelGGL(k_rotate<float>, dim3(blocks), dim3(256), 0, st, d, mu, phi, out, n);
    else hipLaunchKernelGGL(k_rotate<double>, dim3(blocks), dim3(256), 0, st, d, mu, phi, out, n);
    return hipGetLastError();
}

}  // namespace mcrt
