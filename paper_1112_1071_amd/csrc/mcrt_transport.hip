// mcrt_transport.hip -- photon-packet transport for gfx950 (Robitaille 2011,
// Sec. 2.2 propagation, Sec. 2.3 Eq. 2 Lucy estimator, Sec. 2.6.1 binning).
//
// One persistent launch processes a whole pass.  Every lane of a wave64 holds
// one packet in registers.  Lanes that have finished a packet take the next
// packet ids from a global pool counter with one atomic per wave (pool
// refill).  Between events a lane walks the grid one cell per loop trip; a
// wave keeps walking until `defer_lanes` of its lanes wait for an event, and
// then handles all waiting lanes of one event type together (event-type
// compaction by ballot), so that the expensive event code runs for many lanes
// at once instead of once per diverging lane.
//
// Per cell crossing a lane reads the cell density (one random gather) and
// adds weight*l*kappa to the cell's FP64 absorption tally with a hardware
// FP64 atomic.  The same template serves the FP64 path (same random stream,
// same decisions as the CPU oracle) and the FP32 transport form.
#include <math.h>

#include "mcrt_internal.h"

namespace mcrt {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror & Shaw 2011): counter (call, 0, packet
// low, packet high), key (seed, pass).  One call yields two uniforms, from the
// 64-bit words (x0:x1) and (x2:x3).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2,
                                              uint32_t& c3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
}

// FP64: u = (floor(w / 2^12) + 1/2) 2^-52 of the 64-bit word w = hi:lo.
// FP32: the same value truncated to 23 bits plus half a unit: (2 floor(hi/2^9) + 1) 2^-24.
template <typename R> __device__ __forceinline__ R make_uniform(uint32_t hi, uint32_t lo);
template <> __device__ __forceinline__ double make_uniform<double>(uint32_t hi, uint32_t lo) {
    const uint64_t w = ((uint64_t)hi << 32) | lo;
    return ((double)(w >> 12) + 0.5) * 0x1p-52;
}
template <> __device__ __forceinline__ float make_uniform<float>(uint32_t hi, uint32_t) {
    return (float)(((hi >> 9) << 1) | 1u) * 0x1p-24f;
}

template <typename R> struct Stream {
    uint32_t k0, k1, p0, p1;
    uint32_t n;
    uint32_t s0, s1;
    __device__ __forceinline__ R next() {
        if ((n & 1u) == 0u) {
            uint32_t c0 = n >> 1, c1 = 0u, c2 = p0, c3 = p1;
            philox4x32_10(c0, c1, c2, c3, k0, k1);
            s0 = c2;
            s1 = c3;
            ++n;
            return make_uniform<R>(c0, c1);
        }
        ++n;
        return make_uniform<R>(s0, s1);
    }
};

template <typename R> struct Const;
template <> struct Const<double> {
    static constexpr double two_pi = 6.283185307179586476925286766559;
    static __device__ __forceinline__ double inf() { return __builtin_inf(); }
};
template <> struct Const<float> {
    static constexpr float two_pi = 6.283185307179586476925286766559f;
    static __device__ __forceinline__ float inf() { return __builtin_inff(); }
};

__device__ __forceinline__ void sin_cos(double x, double* s, double* c) { sincos(x, s, c); }
__device__ __forceinline__ void sin_cos(float x, float* s, float* c) { sincosf(x, s, c); }

// smallest k with u < cdf[k] (cdf[n-1] == 1)
template <typename R>
__device__ __forceinline__ int cdf_search(const R* __restrict__ cdf, int n, R u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

enum : int { ST_EMPTY = 0, ST_WALK = 1, ST_EVENT = 2, ST_ESC = 3, ST_DONE = 4 };

template <typename R> struct Packet {
    int c0, c1, c2;      // cell
    R f0, f1, f2;        // position inside the cell, in cell units [0,1]
    R d0, d1, d2;        // direction (unit vector)
    R is0, is1, is2;     // dx_a / |d_a|
    R tau, tau_acc;      // sampled optical depth and the part used so far
    R chi, kap, wgt;     // opacity of the bin; packet weight (energy / eps0)
    int k;               // frequency bin
    uint32_t nev;        // interactions so far
    uint32_t nlog;       // logged events so far
    uint64_t id;
    int st;
};

template <typename R>
__device__ __forceinline__ void set_direction(Packet<R>& s, const TransportParams<R>& P) {
    s.is0 = P.dxr[0] / fabs(s.d0);
    s.is1 = P.dxr[1] / fabs(s.d1);
    s.is2 = P.dxr[2] / fabs(s.d2);
}

template <typename R>
__device__ __forceinline__ void isotropic(Packet<R>& s, R u_mu, R u_phi) {
    const R mu = (R)2 * u_mu - (R)1;
    const R phi = Const<R>::two_pi * u_phi;
    const R st = sqrt(fmax((R)0, (R)1 - mu * mu));
    R sp, cp;
    sin_cos(phi, &sp, &cp);
    s.d0 = st * cp;
    s.d1 = st * sp;
    s.d2 = mu;
}

// Henyey-Greenstein: inverse cumulative distribution of cos(theta)
template <typename R> __device__ __forceinline__ R hg_mu(R g, R u) {
    R mu;
    if (fabs(g) < (R)1e-6) {
        mu = (R)2 * u - (R)1;
    } else {
        const R f = ((R)1 - g * g) / ((R)1 - g + (R)2 * g * u);
        mu = ((R)1 + g * g - f * f) / ((R)2 * g);
    }
    return fmin((R)1, fmax((R)-1, mu));
}

// new direction at angle acos(mu) from d, azimuth phi about d; renormalised
template <typename R> __device__ __forceinline__ void rotate(Packet<R>& s, R mu, R phi) {
    const R st = sqrt(fmax((R)0, (R)1 - mu * mu));
    R sp, cp;
    sin_cos(phi, &sp, &cp);
    R o0, o1, o2;
    if (fabs(s.d2) > (R)1 - (R)1e-10) {
        const R sgn = s.d2 > (R)0 ? (R)1 : (R)-1;
        o0 = st * cp;
        o1 = st * sp;
        o2 = sgn * mu;
    } else {
        const R q = sqrt((R)1 - s.d2 * s.d2);
        o0 = st * (s.d0 * s.d2 * cp - s.d1 * sp) / q + s.d0 * mu;
        o1 = st * (s.d1 * s.d2 * cp + s.d0 * sp) / q + s.d1 * mu;
        o2 = -st * cp * q + s.d2 * mu;
    }
    const R nrm = sqrt(o0 * o0 + o1 * o1 + o2 * o2);
    s.d0 = o0 / nrm;
    s.d1 = o1 / nrm;
    s.d2 = o2 / nrm;
}

template <typename R>
__device__ __forceinline__ void log_event(Packet<R>& s, const TransportParams<R>& P, int type,
                                          int incl) {
    if ((int64_t)s.id >= P.ev_packets) return;
    const uint32_t i = s.nlog++;
    if (i < (uint32_t)P.ev_cap) {
        mcrt_event* e = P.evlog + (size_t)s.id * P.ev_cap + i;
        e->packet = (int64_t)s.id;
        e->index = (int32_t)i;
        e->type = type;
        e->cell[0] = s.c0;
        e->cell[1] = s.c1;
        e->cell[2] = s.c2;
        e->nu = s.k;
        e->incl = incl;
        e->reserved = 0;
    }
    P.evcount[s.id] = (int32_t)(i + 1);
}

template <typename R>
__device__ __forceinline__ void begin_flight(Packet<R>& s, Stream<R>& rs) {
    s.tau = -log(rs.next());
    s.tau_acc = (R)0;
}

template <typename R>
__device__ __forceinline__ void emit(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                     uint64_t id) {
    s.id = id;
    const uint64_t gid = P.packet_base + id;
    rs.p0 = (uint32_t)gid;
    rs.p1 = (uint32_t)(gid >> 32);
    rs.n = 0;
    const R u_src = rs.next(), u_nu = rs.next(), u_mu = rs.next(), u_phi = rs.next();
    int src;
    if (P.sampling == 0) {
        src = cdf_search(P.lcdf, P.nsrc, u_src);
        s.wgt = (R)1;
    } else {
        src = (int)(gid % (uint64_t)P.nsrc);
        s.wgt = (R)P.sweight[src];
    }
    s.k = cdf_search(P.scdf + (size_t)src * P.nnu, P.nnu, u_nu);
    isotropic(s, u_mu, u_phi);
    set_direction(s, P);
    // start cell: floor of the position in cell units; a position exactly on a
    // wall belongs to the lower cell when the direction is negative on that axis
    const double* x = P.spos + 3 * src;
    {
        double fp = (x[0] - P.lo[0]) / P.dx[0];
        double fl = floor(fp);
        s.c0 = (int)fl;
        s.f0 = (R)(fp - fl);
        if (fp == fl && s.d0 < (R)0) { s.c0 -= 1; s.f0 = (R)1; }
        fp = (x[1] - P.lo[1]) / P.dx[1];
        fl = floor(fp);
        s.c1 = (int)fl;
        s.f1 = (R)(fp - fl);
        if (fp == fl && s.d1 < (R)0) { s.c1 -= 1; s.f1 = (R)1; }
        fp = (x[2] - P.lo[2]) / P.dx[2];
        fl = floor(fp);
        s.c2 = (int)fl;
        s.f2 = (R)(fp - fl);
        if (fp == fl && s.d2 < (R)0) { s.c2 -= 1; s.f2 = (R)1; }
    }
    s.chi = P.chi[s.k];
    s.kap = P.kap[s.k];
    s.nev = 0;
    s.nlog = 0;
    log_event(s, P, MCRT_EV_EMIT, -1);
    begin_flight(s, rs);
    const bool inside = s.c0 >= 0 && s.c0 < P.n[0] && s.c1 >= 0 && s.c1 < P.n[1] && s.c2 >= 0 &&
                        s.c2 < P.n[2];
    s.st = inside ? ST_WALK : ST_ESC;
}

// One segment of the grid walk: to the nearest wall, or to the interaction
// point if the sampled optical depth is used up inside this cell.
template <typename R>
__device__ __forceinline__ void step(Packet<R>& s, const TransportParams<R>& P, uint32_t* cnt) {
    const R INF = Const<R>::inf();
    const int j = s.c0 + P.n[0] * (s.c1 + P.n[1] * s.c2);
    const R t0 = s.d0 > (R)0 ? ((R)1 - s.f0) * s.is0 : (s.d0 < (R)0 ? s.f0 * s.is0 : INF);
    const R t1 = s.d1 > (R)0 ? ((R)1 - s.f1) * s.is1 : (s.d1 < (R)0 ? s.f1 * s.is1 : INF);
    const R t2 = s.d2 > (R)0 ? ((R)1 - s.f2) * s.is2 : (s.d2 < (R)0 ? s.f2 * s.is2 : INF);
    int ax = 0;
    R tm = t0;
    if (t1 < tm) { ax = 1; tm = t1; }
    if (t2 < tm) { ax = 2; tm = t2; }
    R l = fmax(tm, (R)0);
    const R rho = P.rho[j];
    bool interact = false;
    if (rho > (R)0) {
        ++cnt[C_CROSS_DUST];
        const R rc = rho * s.chi;
        const R dtau = rc * l;
        if (s.tau_acc + dtau >= s.tau) {
            l = (s.tau - s.tau_acc) / rc;
            interact = true;
        } else {
            s.tau_acc += dtau;
        }
        const R w = s.wgt * l * s.kap;
        unsafeAtomicAdd(P.acc + j, (double)w);
        if (P.acc2) unsafeAtomicAdd(P.acc2 + j, (double)w * (double)w);
    } else {
        ++cnt[C_CROSS_EMPTY];
    }
    const R a0 = s.f0 + s.d0 * P.inv_dx[0] * l;
    const R a1 = s.f1 + s.d1 * P.inv_dx[1] * l;
    const R a2 = s.f2 + s.d2 * P.inv_dx[2] * l;
    if (interact) {
        s.f0 = fmin((R)1, fmax((R)0, a0));
        s.f1 = fmin((R)1, fmax((R)0, a1));
        s.f2 = fmin((R)1, fmax((R)0, a2));
        s.st = ST_EVENT;
        return;
    }
    s.f0 = fmin((R)1, fmax((R)0, a0));
    s.f1 = fmin((R)1, fmax((R)0, a1));
    s.f2 = fmin((R)1, fmax((R)0, a2));
    if (ax == 0) {
        const bool up = s.d0 > (R)0;
        const int cn = s.c0 + (up ? 1 : -1);
        if (cn < 0 || cn >= P.n[0]) { s.f0 = up ? (R)1 : (R)0; s.st = ST_ESC; }
        else { s.c0 = cn; s.f0 = up ? (R)0 : (R)1; }
    } else if (ax == 1) {
        const bool up = s.d1 > (R)0;
        const int cn = s.c1 + (up ? 1 : -1);
        if (cn < 0 || cn >= P.n[1]) { s.f1 = up ? (R)1 : (R)0; s.st = ST_ESC; }
        else { s.c1 = cn; s.f1 = up ? (R)0 : (R)1; }
    } else {
        const bool up = s.d2 > (R)0;
        const int cn = s.c2 + (up ? 1 : -1);
        if (cn < 0 || cn >= P.n[2]) { s.f2 = up ? (R)1 : (R)0; s.st = ST_ESC; }
        else { s.c2 = cn; s.f2 = up ? (R)0 : (R)1; }
    }
}

// Scatter (u <= albedo) or absorb and re-emit (Sec. 2.2), then a new flight.
template <typename R>
__device__ __forceinline__ void interact(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                         uint32_t* cnt, double& e_killed) {
    s.nev += 1;
    if ((int64_t)s.nev > P.max_events) {
        ++cnt[C_KILLED];
        e_killed += P.eps0 * (double)s.wgt;
        log_event(s, P, MCRT_EV_KILLED, -1);
        s.st = ST_EMPTY;
        return;
    }
    const R u_int = rs.next();
    if (u_int > P.alb[s.k]) {
        const R u_mix = rs.next(), u_nu = rs.next(), u_mu = rs.next(), u_phi = rs.next();
        const int j = s.c0 + P.n[0] * (s.c1 + P.n[1] * s.c2);
        const R p = P.rowpos[j];
        int m = (int)p;
        m = m > kRows - 2 ? kRows - 2 : m;
        const R w = p - (R)m;
        const int row = m + (u_mix < w ? 1 : 0);
        s.k = cdf_search(P.ecdf + (size_t)row * P.nnu, P.nnu, u_nu);
        isotropic(s, u_mu, u_phi);
        ++cnt[C_ABSORB];
        log_event(s, P, MCRT_EV_ABSORB, -1);
        s.chi = P.chi[s.k];
        s.kap = P.kap[s.k];
    } else {
        const R u_mu = rs.next(), u_phi = rs.next();
        const R mu = hg_mu(P.g[s.k], u_mu);
        rotate(s, mu, Const<R>::two_pi * u_phi);
        ++cnt[C_SCATTER];
        log_event(s, P, MCRT_EV_SCATTER, -1);
    }
    set_direction(s, P);
    begin_flight(s, rs);
    s.st = ST_WALK;
}

template <typename R>
__device__ __forceinline__ void escape(Packet<R>& s, const TransportParams<R>& P, uint32_t* cnt,
                                       double& e_escaped) {
    const R fz = fmin((R)P.n_incl, fmax((R)0, fabs(s.d2) * (R)P.n_incl));  // NaN -> 0
    int incl = (int)fz;
    incl = incl >= P.n_incl ? P.n_incl - 1 : incl;
    const double eps = P.eps0 * (double)s.wgt;
    ++cnt[C_ESCAPE];
    e_escaped += eps;
    if (P.binning) {
        const size_t q = (size_t)incl * P.nnu + s.k;
        unsafeAtomicAdd(P.sed_sum + q, eps);
        unsafeAtomicAdd(P.sed_sum2 + q, eps * eps);
        atomicAdd(P.sed_n + q, 1ull);
        const int ii = P.n_img > 0 ? P.img_of_bin[s.k] : -1;
        if (ii >= 0) {
            // project the escape point on the plane perpendicular to d
            const double px = P.lo[0] + ((double)s.c0 + (double)s.f0) * P.dx[0] -
                              (P.lo[0] + 0.5 * P.n[0] * P.dx[0]);
            const double py = P.lo[1] + ((double)s.c1 + (double)s.f1) * P.dx[1] -
                              (P.lo[1] + 0.5 * P.n[1] * P.dx[1]);
            const double pz = P.lo[2] + ((double)s.c2 + (double)s.f2) * P.dx[2] -
                              (P.lo[2] + 0.5 * P.n[2] * P.dx[2]);
            const double d0 = s.d0, d1 = s.d1, d2 = s.d2;
            double ex0 = -d1, ex1 = d0;
            const double en = sqrt(ex0 * ex0 + ex1 * ex1);
            if (en < 1e-12) { ex0 = 1.0; ex1 = 0.0; }
            else { ex0 /= en; ex1 /= en; }
            // e_y = d x e_x with e_x = (ex0, ex1, 0)
            const double ey0 = -d2 * ex1, ey1 = d2 * ex0, ey2 = d0 * ex1 - d1 * ex0;
            const double X = px * ex0 + py * ex1;
            const double Y = px * ey0 + py * ey1 + pz * ey2;
            const double fx = floor((X + P.img_hw) / (2.0 * P.img_hw) * P.npix);
            const double fy = floor((Y + P.img_hw) / (2.0 * P.img_hw) * P.npix);
            if (fx >= 0.0 && fy >= 0.0 && fx < P.npix && fy < P.npix) {
                const size_t q2 = (((size_t)ii * P.n_incl + incl) * P.npix + (size_t)fy) * P.npix +
                                  (size_t)fx;
                unsafeAtomicAdd(P.img_sum + q2, eps);
                unsafeAtomicAdd(P.img_sum2 + q2, eps * eps);
            }
        }
    }
    log_event(s, P, MCRT_EV_ESCAPE, incl);
    s.st = ST_EMPTY;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = __shfl((int)(uint32_t)v, src);
    const uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

template <typename R>
__global__ void __launch_bounds__(256) k_transport(TransportParams<R> P) {
    __shared__ unsigned long long s_cnt[C_COUNT];
    __shared__ double s_energy[2];
    if (threadIdx.x < C_COUNT) s_cnt[threadIdx.x] = 0ull;
    if (threadIdx.x < 2) s_energy[threadIdx.x] = 0.0;
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

    for (;;) {
        // pool refill: one atomic per wave hands consecutive ids to the empty lanes
        const unsigned long long need = __ballot(s.st == ST_EMPTY);
        if (need) {
            const int leader = __ffsll((long long)need) - 1;
            unsigned long long base = 0;
            if (lane == leader) base = atomicAdd(P.pool, (unsigned long long)__popcll(need));
            base = shfl_u64(base, leader);
            if (s.st == ST_EMPTY) {
                const uint64_t my = base + __popcll(need & __lanemask_lt());
                if (my < P.n_packets) emit(s, rs, P, my);
                else s.st = ST_DONE;
            }
        }
        if (__ballot(s.st != ST_DONE) == 0ull) break;
        // walk until enough lanes wait for an event (or none walks)
        for (;;) {
            if (s.st == ST_WALK) step(s, P, cnt);
            if (__ballot(s.st == ST_WALK) == 0ull) break;
            if (__popcll(__ballot(s.st == ST_EVENT || s.st == ST_ESC)) >= defer) break;
        }
        if (s.st == ST_EVENT) interact(s, rs, P, cnt, e_killed);
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

template <typename R>
hipError_t launch_transport(const TransportParams<R>& P, int blocks, int threads, hipStream_t st) {
    hipLaunchKernelGGL(k_transport<R>, dim3(blocks), dim3(threads), 0, st, P);
    return hipGetLastError();
}

template <typename R> int transport_max_blocks_per_cu(int threads) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_transport<R>, threads, 0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template hipError_t launch_transport<double>(const TransportParams<double>&, int, int, hipStream_t);
template hipError_t launch_transport<float>(const TransportParams<float>&, int, int, hipStream_t);
template int transport_max_blocks_per_cu<double>(int);
template int transport_max_blocks_per_cu<float>(int);

}  // namespace mcrt
