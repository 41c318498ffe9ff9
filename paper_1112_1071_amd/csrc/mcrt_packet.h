// mcrt_packet.h -- device-side state and steps of one photon packet, shared
// by the transport kernels (per-lane persistent walk and tiled sweeps):
// random streams, emission (Sec. 2.1.1), flights and the grid walk with the
// Lucy estimator (Sec. 2.2, Sec. 2.3 Eq. 2), scattering and absorption with
// re-emission (Sec. 2.2), escape and binning (Sec. 2.6.1).
#pragma once
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
        // each 32 x 32 -> 64-bit product in one multiply, both halves used
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
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

// Uniform n of a packet's stream is half of Philox block n / 2: the first
// pair of words for even n, the second for odd n.  The second pair is kept
// from the block's call; s0 = s1 = 0 marks it as not kept (a stream restored
// from a stored position), and the block is then computed again when the
// pair is drawn: the same block gives the same words, so a pair that is
// really zero costs one recomputation and nothing else.
template <typename R> struct Stream {
    uint32_t k0, k1, p0, p1;
    uint32_t n;
    uint32_t s0, s1;
    __device__ __forceinline__ R next() {
        const bool first = (n & 1u) == 0u;
        if (first || (s0 | s1) == 0u) {
            uint32_t c0 = n >> 1, c1 = 0u, c2 = p0, c3 = p1;
            philox4x32_10(c0, c1, c2, c3, k0, k1);
            s0 = c2;
            s1 = c3;
            ++n;
            return first ? make_uniform<R>(c0, c1) : make_uniform<R>(c2, c3);
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

// smallest k with u < cdf[k] (cdf[n-1] == 1), plain binary search
template <typename R>
__device__ __forceinline__ int cdf_search(const R* cdf, int n, R u) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < cdf[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// number of entries <= u among the 16 entries of a group (64 B of FP32, 128 B of FP64)
__device__ __forceinline__ int count_le16(const float* __restrict__ g, float u) {
    const float4* v = reinterpret_cast<const float4*>(g);
    int c = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const float4 q = v[i];
        c += (q.x <= u) + (q.y <= u) + (q.z <= u) + (q.w <= u);
    }
    return c;
}
__device__ __forceinline__ int count_le16(const double* __restrict__ g, double u) {
    const double2* v = reinterpret_cast<const double2*>(g);
    int c = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 q = v[i];
        c += (q.x <= u) + (q.y <= u);
    }
    return c;
}

// Same result as cdf_search on a padded row: the coarse index (every 16th
// entry, usually in LDS) selects the group, one group read finishes it.
template <typename R>
__device__ __forceinline__ int cdf_search2(const R* row, const R* coarse, int ngroup, R u) {
    int lo = 0, hi = ngroup - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u < coarse[mid]) hi = mid;
        else lo = mid + 1;
    }
    return kGroup * lo + count_le16(row + kGroup * lo, u);
}

enum : int { ST_EMPTY = 0, ST_WALK = 1, ST_EVENT = 2, ST_ESC = 3, ST_DONE = 4 };

template <typename R> struct Packet {
    int c0, c1, c2;      // current cell
    R d0, d1, d2;        // direction (unit vector)
    R u0, u1, u2;        // flight origin in grid cell units (cell index + in-cell offset)
    R tx, ty, tz;        // ray distance from the flight origin to the next wall per axis
    R dtx, dty, dtz;     // ray distance between walls per axis: dx_a / |d_a|
    R t;                 // ray distance walked in this flight
    R tau, tau_acc;      // sampled optical depth and the part used so far
    R chi, kap, wgt;     // opacity of the bin; packet weight (energy / eps0)
    R rowp;              // emission-row position of the cell of a pending interaction,
                         // when the kernel loads it ahead (tiled sweeps)
    int k;               // frequency bin
    uint32_t nev;        // interactions so far
    uint32_t nlog;       // logged events so far
    uint64_t id;
    int st;
};

template <int BRICK, typename P>
__device__ __forceinline__ int cell_index(const P& p, int c0, int c1, int c2) {
    if (BRICK)
        return ((((c2 >> 2) * p.bxy + (c1 >> 2) * p.bx + (c0 >> 2)) << 6) | ((c2 & 3) << 4) |
                ((c1 & 3) << 2) | (c0 & 3));
    return c0 + p.n[0] * (c1 + p.n[1] * c2);
}

template <int BRICK, typename P>
__device__ __forceinline__ void cell_coords(const P& p, int j, int& c0, int& c1, int& c2) {
    if (BRICK) {
        const int b = j >> 6, o = j & 63;
        const int bz = b / p.bxy, r = b - bz * p.bxy;
        const int by = r / p.bx, bxx = r - by * p.bx;
        c0 = (bxx << 2) | (o & 3);
        c1 = (by << 2) | ((o >> 2) & 3);
        c2 = (bz << 2) | (o >> 4);
    } else {
        const int nxy = p.n[0] * p.n[1];
        c2 = j / nxy;
        const int r = j - c2 * nxy;
        c1 = r / p.n[0];
        c0 = r - c1 * p.n[0];
    }
}

// Start a flight from cell c with in-cell offset f: wall distances per axis,
// then tau = -ln(u) (Sec. 2.2).
template <typename R>
__device__ __forceinline__ void begin_flight(Packet<R>& s, const TransportParams<R>& P,
                                             Stream<R>& rs, R f0, R f1, R f2) {
    const R INF = Const<R>::inf();
    s.u0 = (R)s.c0 + f0;
    s.u1 = (R)s.c1 + f1;
    s.u2 = (R)s.c2 + f2;
    s.dtx = P.dxr[0] / fabs(s.d0);
    s.dty = P.dxr[1] / fabs(s.d1);
    s.dtz = P.dxr[2] / fabs(s.d2);
    s.tx = s.d0 == (R)0 ? INF : (s.d0 > (R)0 ? (R)1 - f0 : f0) * s.dtx;
    s.ty = s.d1 == (R)0 ? INF : (s.d1 > (R)0 ? (R)1 - f1 : f1) * s.dty;
    s.tz = s.d2 == (R)0 ? INF : (s.d2 > (R)0 ? (R)1 - f2 : f2) * s.dtz;
    s.t = (R)0;
    s.tau = -log(rs.next());
    s.tau_acc = (R)0;
}

// in-cell offset of the point at ray distance t of the current flight
template <typename R>
__device__ __forceinline__ void offsets_at(const Packet<R>& s, const TransportParams<R>& P, R t,
                                           R& f0, R& f1, R& f2) {
    f0 = fmin((R)1, fmax((R)0, s.u0 + s.d0 * P.inv_dx[0] * t - (R)s.c0));
    f1 = fmin((R)1, fmax((R)0, s.u1 + s.d1 * P.inv_dx[1] * t - (R)s.c1));
    f2 = fmin((R)1, fmax((R)0, s.u2 + s.d2 * P.inv_dx[2] * t - (R)s.c2));
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

// New direction at angle acos(mu) from d, azimuth phi about d; renormalised.
// q = |d_perp| = sin(theta_d).  In FP64 q = sqrt(1 - d_z^2) with the pole
// branch for |d_z| > 1 - 1e-10 (the oracle's arithmetic).  In FP32 that test
// cannot work (1 - 1e-10 rounds to 1, and a direction within ~2.4e-4 rad of
// the pole stores d_z = +-1 exactly, giving q = 0), so q is taken from the
// transverse components themselves, sqrt(d_x^2 + d_y^2), which stays accurate
// down to the pole; only d_x = d_y = 0 takes the pole branch.  Packet
// histories must not depend on which kernel walks a packet, so each FP32 sum
// of products here is written as one explicit fused multiply-add.
template <typename R>
__device__ __forceinline__ void rotate_dir(R& d0, R& d1, R& d2, R mu, R phi) {
    const R st = sqrt(fmax((R)0, (R)1 - mu * mu));
    R sp, cp;
    sin_cos(phi, &sp, &cp);
    R q;
    bool pole;
    if constexpr (sizeof(R) == 8) {
        pole = fabs(d2) > (R)1 - (R)1e-10;
        q = pole ? (R)1 : sqrt((R)1 - d2 * d2);
    } else {
        // one explicit fused multiply-add, so that every kernel rounds alike
        q = sqrt(fmaf(d0, d0, d1 * d1));
        pole = !(q > (R)1e-30);
    }
    R o0, o1, o2;
    if (pole) {
        const R sgn = d2 > (R)0 ? (R)1 : (R)-1;
        o0 = st * cp;
        o1 = st * sp;
        o2 = sgn * mu;
    } else {
        o0 = st * (d0 * d2 * cp - d1 * sp) / q + d0 * mu;
        o1 = st * (d1 * d2 * cp + d0 * sp) / q + d1 * mu;
        o2 = -st * cp * q + d2 * mu;
    }
    const R nrm = sqrt(o0 * o0 + o1 * o1 + o2 * o2);
    d0 = o0 / nrm;
    d1 = o1 / nrm;
    d2 = o2 / nrm;
}

template <typename R> __device__ __forceinline__ void rotate(Packet<R>& s, R mu, R phi) {
    rotate_dir(s.d0, s.d1, s.d2, mu, phi);
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

// Tables the event code reads (from LDS where a kernel staged them): the
// luminosity CDF, the coarse indices of the emission and source-spectrum CDFs,
// and the dust properties per bin.
template <typename R> struct Tables {
    const R* lcdf;
    const R* ecoarse;
    const R* scoarse;
    const R* chi;
    const R* kap;
    const R* alb;
    const R* g;
};

template <typename R> __device__ __forceinline__ Tables<R> global_tables(const TransportParams<R>& P) {
    return Tables<R>{P.lcdf, P.ecoarse, P.scoarse, P.chi, P.kap, P.alb, P.g};
}

// Optical depth in bin k from the point (cell c, in-cell offsets f) to the
// grid boundary along the unit vector o: the walk of a flight, without
// interactions, on the x-fastest density.
template <typename R>
__device__ double tau_to_boundary(const TransportParams<R>& P, int c0, int c1, int c2, R f0, R f1,
                                  R f2, double o0, double o1, double o2, R chi) {
    const R INF = Const<R>::inf();
    const R d0 = (R)o0, d1 = (R)o1, d2 = (R)o2;
    const R dtx = P.dxr[0] / fabs(d0), dty = P.dxr[1] / fabs(d1), dtz = P.dxr[2] / fabs(d2);
    R tx = d0 == (R)0 ? INF : (d0 > (R)0 ? (R)1 - f0 : f0) * dtx;
    R ty = d1 == (R)0 ? INF : (d1 > (R)0 ? (R)1 - f1 : f1) * dty;
    R tz = d2 == (R)0 ? INF : (d2 > (R)0 ? (R)1 - f2 : f2) * dtz;
    R t = (R)0;
    double tau = 0.0;
    // a start point on a wall belongs to the cell the ray enters (the start
    // cell rule of emission, applied with the direction o)
    if (f0 == (R)1 && d0 >= (R)0) { ++c0; f0 = (R)0; tx = d0 == (R)0 ? INF : dtx; }
    else if (f0 == (R)0 && d0 < (R)0) { --c0; f0 = (R)1; tx = dtx; }
    if (f1 == (R)1 && d1 >= (R)0) { ++c1; f1 = (R)0; ty = d1 == (R)0 ? INF : dty; }
    else if (f1 == (R)0 && d1 < (R)0) { --c1; f1 = (R)1; ty = dty; }
    if (f2 == (R)1 && d2 >= (R)0) { ++c2; f2 = (R)0; tz = d2 == (R)0 ? INF : dtz; }
    else if (f2 == (R)0 && d2 < (R)0) { --c2; f2 = (R)1; tz = dtz; }
    if ((unsigned)c0 >= (unsigned)P.n[0] || (unsigned)c1 >= (unsigned)P.n[1] ||
        (unsigned)c2 >= (unsigned)P.n[2])
        return 0.0;
    for (;;) {
        const bool ax1 = ty < tx;
        R tm = ax1 ? ty : tx;
        const bool ax2 = tz < tm;
        tm = ax2 ? tz : tm;
        const bool ax0 = !ax1 && !ax2;
        const bool by = ax1 && !ax2;
        const R l = fmax(tm - t, (R)0);
        tau += (double)(P.rho_lin[c0 + (int64_t)P.n[0] * (c1 + (int64_t)P.n[1] * c2)] * chi * l);
        t = fmax(tm, t);
        c0 += ax0 ? (d0 > (R)0 ? 1 : -1) : 0;
        c1 += by ? (d1 > (R)0 ? 1 : -1) : 0;
        c2 += ax2 ? (d2 > (R)0 ? 1 : -1) : 0;
        if ((unsigned)c0 >= (unsigned)P.n[0] || (unsigned)c1 >= (unsigned)P.n[1] ||
            (unsigned)c2 >= (unsigned)P.n[2])
            return tau;
        tx += ax0 ? dtx : (R)0;
        ty += by ? dty : (R)0;
        tz += ax2 ? dtz : (R)0;
    }
}

// Peeling-off (Sec. 2.6.2): toward every observer o, eps * p(o) * exp(-tau)
// in the packet's bin into SED component comp (0 direct, 1 processed) and,
// for image bins, into the pixel of the packet's position projected along o.
// p is the HG phase function per steradian for the incoming direction
// (scattering, have_din) or 1/(4 pi) for isotropic emission.
template <typename R>
__device__ void peel(const Packet<R>& s, const TransportParams<R>& P, R f0, R f1, R f2, int comp,
                     bool have_din, double di0, double di1, double di2) {
    const double four_pi = 12.566370614359172953850573533118;
    const double g = (double)P.g[s.k];
    const double eps = P.eps0 * (double)s.wgt;
    const int ii = P.n_img > 0 ? P.img_of_bin[s.k] : -1;
    for (int i = 0; i < P.n_peel; ++i) {
        const double o0 = P.peel_dir[3 * i], o1 = P.peel_dir[3 * i + 1], o2 = P.peel_dir[3 * i + 2];
        double p = 1.0 / four_pi;
        if (have_din) {
            const double q = 1.0 + g * g - 2.0 * g * (di0 * o0 + di1 * o1 + di2 * o2);
            p = (1.0 - g * g) / (four_pi * q * sqrt(q));
        }
        const double w = eps * p * exp(-tau_to_boundary(P, s.c0, s.c1, s.c2, f0, f1, f2, o0, o1, o2, s.chi));
        const size_t q = ((size_t)i * 2 + comp) * P.nnu + s.k;
        unsafeAtomicAdd(P.psed_sum + q, w);
        unsafeAtomicAdd(P.psed_sum2 + q, w * w);
        if (ii < 0) continue;
        const double px = ((double)s.c0 + (double)f0 - 0.5 * P.n[0]) * P.dx[0];
        const double py = ((double)s.c1 + (double)f1 - 0.5 * P.n[1]) * P.dx[1];
        const double pz = ((double)s.c2 + (double)f2 - 0.5 * P.n[2]) * P.dx[2];
        double ex0 = -o1, ex1 = o0;
        const double en = sqrt(ex0 * ex0 + ex1 * ex1);
        if (en < 1e-12) { ex0 = 1.0; ex1 = 0.0; }
        else { ex0 /= en; ex1 /= en; }
        const double ey0 = -o2 * ex1, ey1 = o2 * ex0, ey2 = o0 * ex1 - o1 * ex0;
        const double X = px * ex0 + py * ex1;
        const double Y = px * ey0 + py * ey1 + pz * ey2;
        const double fx = floor((X + P.img_hw) / (2.0 * P.img_hw) * P.npix);
        const double fy = floor((Y + P.img_hw) / (2.0 * P.img_hw) * P.npix);
        if (fx >= 0.0 && fy >= 0.0 && fx < P.npix && fy < P.npix) {
            const size_t r = (((size_t)ii * P.n_peel + i) * P.npix + (size_t)fy) * P.npix + (size_t)fx;
            unsafeAtomicAdd(P.pimg_sum + r, w);
            unsafeAtomicAdd(P.pimg_sum2 + r, w * w);
        }
    }
}

// Where a modified-random-walk step adds to the absorption tally: the global
// FP64 tally in the per-lane walk's layout, or the tile's LDS tally.
template <int BRICK> struct GlobalDeposit {
    double* acc;
    double* acc2;
    int n[3];
    int bx, bxy;
    template <typename R> __device__ void operator()(int c0, int c1, int c2, R w) const {
        const int j = cell_index<BRICK>(*this, c0, c1, c2);
        unsafeAtomicAdd(acc + j, (double)w);
        if (acc2) unsafeAtomicAdd(acc2 + j, (double)w * (double)w);
    }
};

template <int BRICK, typename R>
__device__ __forceinline__ GlobalDeposit<BRICK> global_deposit(const TransportParams<R>& P, double* acc) {
    return GlobalDeposit<BRICK>{acc, P.acc2, {P.n[0], P.n[1], P.n[2]}, P.bx, P.bxy};
}

// The tile's LDS tally: FP64 sums of the (transport-precision) weights.
template <typename R> struct TileDeposit {
    double* acc;
    double* acc2;
    int o0, o1, o2, txy;
    __device__ void operator()(int c0, int c1, int c2, R w) const {
        const int jl = (c0 - o0) + txy * ((c1 - o1) + txy * (c2 - o2));
        atomicAdd(acc + jl, (double)w);
        if (acc2) atomicAdd(acc2 + jl, (double)w * (double)w);
    }
};

// Re-emission bin from the emissivity of cell j: row m or m+1 of the cell's
// row position (u_mix), then the row's CDF (u_nu).
template <typename R>
__device__ __forceinline__ int reemission_row_bin(const TransportParams<R>& P, const Tables<R>& tb, R p,
                                                  R u_mix, R u_nu) {
    int m = (int)p;
    m = m > kRows - 2 ? kRows - 2 : m;
    const R w = p - (R)m;
    const int row = m + (u_mix < w ? 1 : 0);
    return cdf_search2(P.ecdf + (size_t)row * P.npad, tb.ecoarse + row * P.ngroup, P.ngroup, u_nu);
}

template <typename R>
__device__ __forceinline__ int reemission_bin(const TransportParams<R>& P, const Tables<R>& tb, int64_t j,
                                              R u_mix, R u_nu) {
    return reemission_row_bin(P, tb, P.rowpos[j], u_mix, u_nu);
}

// ---- modified random walk (Sec. 2.2) ---------------------------------------
// The paper names the method (with its gamma) without its steps; they follow
// from diffusion in a sphere.  First-passage distribution of diffusion from
// the centre of a sphere, y = pi^2 D t / R^2:
//   F(y) = 1 + 2 sum_{n>=1} (-1)^n exp(-n^2 y)
//        = 2 sqrt(pi/y) sum_{m>=0} exp(-pi^2 (2m+1)^2 / (4y))   (Jacobi),
// the second form for y < 2.
__device__ inline double mrw_cdf(double y) {
    const double pi = 3.14159265358979323846;
    if (!(y > 0.0)) return 0.0;
    double f = 0.0;
    if (y < 2.0) {
        for (int m = 0; m < 40; ++m) {
            const double a = (2 * m + 1) * pi;
            const double t = exp(-a * a / (4.0 * y));
            f += t;
            if (t < 1e-20 * f) break;
        }
        return 2.0 * sqrt(pi / y) * f;
    }
    double sg = -1.0;
    for (int n = 1; n < 40; ++n) {
        const double t = exp(-(double)(n * n) * y);
        f += sg * t;
        sg = -sg;
        if (t < 1e-20) break;
    }
    return 1.0 + 2.0 * f;
}

// y with F(y) = u, by bisection on [1e-3, 80] to the last bit
__device__ inline double mrw_escape_y(double u) {
    double lo = 1e-3, hi = 80.0;
    for (int i = 0; i < 200; ++i) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (mrw_cdf(mid) < u) lo = mid;
        else hi = mid;
    }
    return 0.5 * (lo + hi);
}

// y with F(y) = u from the table of y against w = ln(u / (1 - u)) (values and
// slopes, cubic Hermite; relative error below 1e-10), by bisection outside it
template <typename R>
__device__ inline double mrw_escape_y_tab(const TransportParams<R>& P, double u) {
    const double w = log(u) - log1p(-u);
    const double h = (kMrwW1 - kMrwW0) / (kMrwYRows - 1);
    const double p = (w - kMrwW0) / h;
    if (!(p >= 0.0 && p <= (double)(kMrwYRows - 1))) return mrw_escape_y(u);
    int i = (int)p;
    i = i > kMrwYRows - 2 ? kMrwYRows - 2 : i;
    const double t = p - i, t2 = t * t, t3 = t2 * t;
    const double* a = P.mrw_ytab + 2 * (size_t)i;
    return (2 * t3 - 3 * t2 + 1) * a[0] + (t3 - 2 * t2 + t) * h * a[1] + (-2 * t3 + 3 * t2) * a[2] +
           (t3 - t2) * h * a[3];
}

// Planck-mean kappa and Rosseland-mean chi of cell j at its temperature:
// cubic Hermite interpolation in ln T of the table
template <typename R>
__device__ inline void mrw_opacities(const TransportParams<R>& P, int64_t j, double& kp, double& chir) {
    const double lo = log(kTLo), h = (log(kTHi) - lo) / (kMrwRows - 1);
    double p = (log(P.Tcell[j]) - lo) / h;
    p = fmin(fmax(p, 0.0), (double)(kMrwRows - 1));
    int i = (int)p;
    i = i > kMrwRows - 2 ? kMrwRows - 2 : i;
    const double t = p - i, t2 = t * t, t3 = t2 * t;
    const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t, h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
    const double* a = P.mrw_tab + 4 * (size_t)i;
    const double* b = a + 4;
    kp = h00 * a[0] + h10 * h * a[1] + h01 * b[0] + h11 * h * b[1];
    chir = h00 * a[2] + h10 * h * a[3] + h01 * b[2] + h11 * h * b[3];
}

// Modified-random-walk steps from the in-cell offsets f: while the sphere to
// the nearest cell wall (radius R0) holds at least mrw_gamma Rosseland mean
// free paths, the packet diffuses to a uniformly random point of it over the
// path length s = 3 rho chi_R R0^2 y / pi^2 (y from F), adds w kappa_P s to
// the cell's tally (dep), and is re-emitted from the cell's emissivity in an
// isotropic direction.  Draws u_y u_mu u_phi u_mix u_nu u_mu u_phi per step.
// Returns false when the packet was killed at the event limit.
template <typename R, typename Dep>
__device__ bool mrw_steps(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P, const Tables<R>& tb,
                          R& f0, R& f1, R& f2, uint32_t* cnt, double& e_killed, const Dep& dep) {
    const double pi = 3.14159265358979323846;
    const int64_t j = s.c0 + (int64_t)P.n[0] * (s.c1 + (int64_t)P.n[1] * s.c2);
    const double r = (double)P.rho_lin[j];
    if (!(r > 0.0)) return true;
    double kp, chir;
    mrw_opacities(P, j, kp, chir);
    for (;;) {
        const double g0 = (double)f0 * P.dx[0], g1 = (double)f1 * P.dx[1], g2 = (double)f2 * P.dx[2];
        const double R0 = fmin(fmin(fmin(g0, P.dx[0] - g0), fmin(g1, P.dx[1] - g1)), fmin(g2, P.dx[2] - g2));
        if (!(r * chir * R0 >= P.mrw_gamma)) return true;
        s.nev += 1;
        if ((int64_t)s.nev > P.max_events) {
            ++cnt[C_KILLED];
            e_killed += P.eps0 * (double)s.wgt;
            log_event(s, P, MCRT_EV_KILLED, -1);
            s.st = ST_EMPTY;
            return false;
        }
        const R u_y = rs.next(), u_mu = rs.next(), u_phi = rs.next(), u_mix = rs.next(), u_nu = rs.next();
        const R u_mu2 = rs.next(), u_phi2 = rs.next();
        const double y = mrw_escape_y_tab(P, (double)u_y);
        const double sp = 3.0 * r * chir * R0 * R0 * y / (pi * pi);
        dep(s.c0, s.c1, s.c2, (R)((double)s.wgt * kp * sp));
        const double mu = 2.0 * (double)u_mu - 1.0, phi = 2.0 * pi * (double)u_phi;
        const double st = sqrt(fmax(0.0, 1.0 - mu * mu));
        f0 = (R)fmin(1.0, fmax(0.0, (g0 + R0 * st * cos(phi)) / P.dx[0]));
        f1 = (R)fmin(1.0, fmax(0.0, (g1 + R0 * st * sin(phi)) / P.dx[1]));
        f2 = (R)fmin(1.0, fmax(0.0, (g2 + R0 * mu) / P.dx[2]));
        s.k = reemission_bin(P, tb, j, u_mix, u_nu);
        isotropic(s, u_mu2, u_phi2);
        s.chi = tb.chi[s.k];
        s.kap = tb.kap[s.k];
        ++cnt[C_MRW];
        log_event(s, P, MCRT_EV_MRW, -1);
        if (P.binning && P.n_peel > 0) peel(s, P, f0, f1, f2, 1, false, 0.0, 0.0, 0.0);
    }
}

// First part of an emission (Sec. 2.1.1, 2.2): the packet's stream, its four
// draws u_src u_nu u_mu u_phi, the source (luminosity CDF, or packet id mod
// the number of sources), its weight and isotropic direction, and the start
// cell with the in-cell offsets f: the floor of the position in cell units;
// a position exactly on a wall belongs to the lower cell when the direction is
// negative on that axis.  Returns the source; u_nu is left for the bin.
template <typename R>
__device__ __forceinline__ int emit_start(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                          const Tables<R>& tb, uint64_t id, R& u_nu, R f[3]) {
    s.id = id;
    const uint64_t gid = P.packet_base + id;
    rs.p0 = (uint32_t)gid;
    rs.p1 = (uint32_t)(gid >> 32);
    rs.n = 0;
    const R u_src = rs.next();
    u_nu = rs.next();
    const R u_mu = rs.next(), u_phi = rs.next();
    int src;
    if (P.sampling == 0) {
        src = cdf_search(tb.lcdf, P.nsrc, u_src);
        s.wgt = (R)1;
    } else {
        src = (int)(gid % (uint64_t)P.nsrc);
        s.wgt = (R)P.sweight[src];
    }
    isotropic(s, u_mu, u_phi);
    // the source's cell and offsets, (x - lo) / dx split into its floor and
    // the rest, tabulated per source in FP64
    const int4 sc = P.scell[src];
    const double* fr = P.sfrac + 3 * src;
    int c[3] = {sc.x, sc.y, sc.z};
    const R dd[3] = {s.d0, s.d1, s.d2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f[a] = (R)fr[a];
        if (((sc.w >> a) & 1) && dd[a] < (R)0) {
            c[a] -= 1;
            f[a] = (R)1;
        }
    }
    s.c0 = c[0];
    s.c1 = c[1];
    s.c2 = c[2];
    return src;
}

// The start cell of packet id, as emit_start finds it, from the source's
// tabulated cell: one random block for the source, and the direction only for
// a source on a cell wall, where its sign picks the cell.
template <typename R>
__device__ __forceinline__ void emit_start_cell(Stream<R>& rs, const TransportParams<R>& P,
                                                const Tables<R>& tb, uint64_t id, int& c0, int& c1,
                                                int& c2) {
    const uint64_t gid = P.packet_base + id;
    rs.p0 = (uint32_t)gid;
    rs.p1 = (uint32_t)(gid >> 32);
    rs.n = 0;
    const R u_src = rs.next();
    const int src = P.sampling == 0 ? cdf_search(tb.lcdf, P.nsrc, u_src) : (int)(gid % (uint64_t)P.nsrc);
    const int4 sc = P.scell[src];
    c0 = sc.x;
    c1 = sc.y;
    c2 = sc.z;
    if (sc.w) {
        rs.next();  // the frequency's uniform
        const R u_mu = rs.next(), u_phi = rs.next();
        Packet<R> s;
        isotropic(s, u_mu, u_phi);
        if ((sc.w & 1) && s.d0 < (R)0) c0 -= 1;
        if ((sc.w & 2) && s.d1 < (R)0) c1 -= 1;
        if ((sc.w & 4) && s.d2 < (R)0) c2 -= 1;
    }
}

template <typename R>
__device__ __forceinline__ bool in_grid(const TransportParams<R>& P, int c0, int c1, int c2) {
    return (unsigned)c0 < (unsigned)P.n[0] && (unsigned)c1 < (unsigned)P.n[1] &&
           (unsigned)c2 < (unsigned)P.n[2];
}

// Emission of packet id: emit_start, the frequency bin from the source's
// spectrum, the log, peeling-off of a binning pass, the modified random walk,
// and the first flight (state WALK inside the grid, ESC outside it; EMPTY if
// the walk killed it).  FULL = false leaves out logging, peeling and the walk
// (a pass that uses none of them).
template <typename R, typename Dep, bool FULL = true>
__device__ __forceinline__ void emit(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                     const Tables<R>& tb, uint64_t id, uint32_t* cnt, double& e_killed,
                                     const Dep& dep) {
    R u_nu;
    R f[3];
    const int src = emit_start(s, rs, P, tb, id, u_nu, f);
    s.k = cdf_search2(P.scdf + (size_t)src * P.npad, tb.scoarse + (size_t)src * P.ngroup, P.ngroup,
                      u_nu);
    s.chi = tb.chi[s.k];
    s.kap = tb.kap[s.k];
    s.nev = 0;
    s.nlog = 0;
    if (FULL) log_event(s, P, MCRT_EV_EMIT, -1);
    if (FULL && P.binning && P.n_peel > 0) peel(s, P, f[0], f[1], f[2], 0, false, 0.0, 0.0, 0.0);
    const bool inside = in_grid(P, s.c0, s.c1, s.c2);
    if (FULL && inside && P.mrw_gamma > 0.0 && !mrw_steps(s, rs, P, tb, f[0], f[1], f[2], cnt, e_killed, dep))
        return;  // killed (s.st = ST_EMPTY)
    begin_flight(s, P, rs, f[0], f[1], f[2]);
    s.st = inside ? ST_WALK : ST_ESC;
}

// K segments of the grid walk: step K walls ahead, gather K densities at
// once, then consume the segments until the optical depth is used up.
// Grid fields the walk reads, held in registers by the batched kernel (whose
// lanes may belong to different models) instead of re-read from memory.
template <typename R> struct WalkGrid {
    int n[3];
    int bx, bxy;
    const R* rho;
    double* acc2;
};

template <typename R, int K, int BRICK, typename G>
__device__ __forceinline__ void walk(Packet<R>& s, const G& P, double* acc, uint32_t* cnt) {
    int jj[K];
    R ll[K], ts[K];
    int nseg = 0;
    bool esc = false;
    const int j0 = cell_index<BRICK>(P, s.c0, s.c1, s.c2);
    int jc = j0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        jj[i] = j0;
        ll[i] = (R)0;
        ts[i] = s.t;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (!esc) {
            // nearest wall; ties go to the lowest axis
            const bool ax1 = s.ty < s.tx;
            R tm = ax1 ? s.ty : s.tx;
            const bool ax2 = s.tz < tm;
            tm = ax2 ? s.tz : tm;
            const bool ax0 = !ax1 && !ax2;
            const bool by = ax1 && !ax2;
            jj[i] = jc;
            ts[i] = s.t;
            ll[i] = fmax(tm - s.t, (R)0);
            nseg = i + 1;
            s.t = fmax(tm, s.t);
            const int n0 = s.c0 + (ax0 ? (s.d0 > (R)0 ? 1 : -1) : 0);
            const int n1 = s.c1 + (by ? (s.d1 > (R)0 ? 1 : -1) : 0);
            const int n2 = s.c2 + (ax2 ? (s.d2 > (R)0 ? 1 : -1) : 0);
            const bool out = (unsigned)n0 >= (unsigned)P.n[0] || (unsigned)n1 >= (unsigned)P.n[1] ||
                             (unsigned)n2 >= (unsigned)P.n[2];
            if (out) {
                esc = true;
            } else {
                s.c0 = n0;
                s.c1 = n1;
                s.c2 = n2;
                s.tx += ax0 ? s.dtx : (R)0;
                s.ty += by ? s.dty : (R)0;
                s.tz += ax2 ? s.dtz : (R)0;
                jc = cell_index<BRICK>(P, n0, n1, n2);
            }
        }
    }
    R rr[K];
#pragma unroll
    for (int i = 0; i < K; ++i) rr[i] = P.rho[jj[i]];
    bool hit = false;
    int jhit = j0;
    R thit = (R)0;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        if (i < nseg && !hit) {
            const R rho = rr[i];
            if (rho > (R)0) {
                ++cnt[C_CROSS_DUST];
                const R rc = rho * s.chi;
                R l = ll[i];
                const R dtau = rc * l;
                if (s.tau_acc + dtau >= s.tau) {
                    l = (s.tau - s.tau_acc) / rc;
                    hit = true;
                    jhit = jj[i];
                    thit = ts[i] + l;
                } else {
                    s.tau_acc += dtau;
                }
                const R w = s.wgt * s.kap * l;  // the tiled walk's order: (wgt kappa) l
                unsafeAtomicAdd(acc + jj[i], (double)w);
                if (P.acc2) unsafeAtomicAdd(P.acc2 + jj[i], (double)w * (double)w);
            } else {
                ++cnt[C_CROSS_EMPTY];
            }
        }
    }
    if (hit) {
        cell_coords<BRICK>(P, jhit, s.c0, s.c1, s.c2);
        s.t = thit;
        s.st = ST_EVENT;
    } else if (esc) {
        s.st = ST_ESC;
    }
}

// Scatter (u <= albedo) or absorb and re-emit (Sec. 2.2), then a new flight.
// PRE: the cell's emission-row position was loaded ahead into s.rowp.
template <typename R, typename Dep, bool FULL = true, bool PRE = false>
__device__ __forceinline__ void interact(Packet<R>& s, Stream<R>& rs, const TransportParams<R>& P,
                                         const Tables<R>& tb, uint32_t* cnt, double& e_killed,
                                         const Dep& dep) {
    s.nev += 1;
    if ((int64_t)s.nev > P.max_events) {
        ++cnt[C_KILLED];
        e_killed += P.eps0 * (double)s.wgt;
        if (FULL) log_event(s, P, MCRT_EV_KILLED, -1);
        s.st = ST_EMPTY;
        return;
    }
    R f0, f1, f2;
    offsets_at(s, P, s.t, f0, f1, f2);
    const R u_int = rs.next();
    if (u_int > tb.alb[s.k]) {
        const R u_mix = rs.next(), u_nu = rs.next(), u_mu = rs.next(), u_phi = rs.next();
        const int64_t j = s.c0 + (int64_t)P.n[0] * (s.c1 + (int64_t)P.n[1] * s.c2);
        s.k = reemission_row_bin(P, tb, PRE ? s.rowp : P.rowpos[j], u_mix, u_nu);
        isotropic(s, u_mu, u_phi);
        ++cnt[C_ABSORB];
        if (FULL) log_event(s, P, MCRT_EV_ABSORB, -1);
        s.chi = tb.chi[s.k];
        s.kap = tb.kap[s.k];
        if (FULL && P.binning && P.n_peel > 0) peel(s, P, f0, f1, f2, 1, false, 0.0, 0.0, 0.0);
    } else {
        const R u_mu = rs.next(), u_phi = rs.next();
        const R mu = hg_mu(tb.g[s.k], u_mu);
        if (FULL && P.binning && P.n_peel > 0) peel(s, P, f0, f1, f2, 1, true, s.d0, s.d1, s.d2);
        rotate(s, mu, Const<R>::two_pi * u_phi);
        ++cnt[C_SCATTER];
        if (FULL) log_event(s, P, MCRT_EV_SCATTER, -1);
    }
    if (FULL && P.mrw_gamma > 0.0 && !mrw_steps(s, rs, P, tb, f0, f1, f2, cnt, e_killed, dep)) return;
    begin_flight(s, P, rs, f0, f1, f2);
    s.st = ST_WALK;
}

template <typename R, bool FULL = true>
__device__ __forceinline__ void escape(Packet<R>& s, const TransportParams<R>& P, uint32_t* cnt,
                                       double& e_escaped) {
    const R fz = fmin((R)P.n_incl, fmax((R)0, fabs(s.d2) * (R)P.n_incl));  // NaN -> 0
    int incl = (int)fz;
    incl = incl >= P.n_incl ? P.n_incl - 1 : incl;
    const double eps = P.eps0 * (double)s.wgt;
    ++cnt[C_ESCAPE];
    e_escaped += eps;
    if (FULL && P.binning) {
        const size_t q = (size_t)incl * P.nnu + s.k;
        unsafeAtomicAdd(P.sed_sum + q, eps);
        unsafeAtomicAdd(P.sed_sum2 + q, eps * eps);
        atomicAdd(P.sed_n + q, 1ull);
        const int ii = P.n_img > 0 ? P.img_of_bin[s.k] : -1;
        if (ii >= 0) {
            // escape point (on the grid boundary), projected on the plane
            // perpendicular to d
            R f0, f1, f2;
            offsets_at(s, P, s.t, f0, f1, f2);
            const double px = ((double)s.c0 + (double)f0 - 0.5 * P.n[0]) * P.dx[0];
            const double py = ((double)s.c1 + (double)f1 - 0.5 * P.n[1]) * P.dx[1];
            const double pz = ((double)s.c2 + (double)f2 - 0.5 * P.n[2]) * P.dx[2];
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
    if (FULL) log_event(s, P, MCRT_EV_ESCAPE, incl);
    s.st = ST_EMPTY;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
    const uint32_t lo = __shfl((int)(uint32_t)v, src);
    const uint32_t hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

}  // namespace mcrt
