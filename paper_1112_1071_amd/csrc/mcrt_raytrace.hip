// mcrt_raytrace.hip -- raytracing of the source and dust emission toward the
// peel-off observers (Sec. 2.6.3), in post-processing at fixed temperatures.
//
// Dust: one wavefront per image pixel.  The wave follows the ray through the
// pixel centre from the observer's side of the grid along -o, cell by cell (a
// DDA on the ray parameter), and its lanes hold the frequency bins (up to 256
// per walk, four per lane): a lane adds exp(-tau in front) S (1 - exp(-dtau)) for
// each of its bins, with
// dtau = rho chi l over the cell's chord l and S = kappa/chi B(T), the bin
// integral of the Planck function read from a per-bin table of ln B in ln T
// (2048 rows over 1..1e4 K, values and slopes, cubic Hermite: relative error
// below about 1e-12 x, x = h nu / k T of the bin) or, outside the table's
// range, taken by composite 4-point Gauss-Legendre quadrature in x.  All lanes of a wave walk the same cells, so the
// walk is uniform control flow and the density and temperature loads are
// broadcasts; bins are the only divergent quantity, and they are the lanes.
// Sources: one wave per (observer, source), optical depth per bin from the
// source to the grid boundary along o.
#include <math.h>

#include "mcrt_internal.h"

namespace mcrt {

namespace {

constexpr double kH = 6.62607015e-27;   // erg s
constexpr double kKB = 1.380649e-16;    // erg / K
constexpr double kC = 2.99792458e10;    // cm / s
constexpr double kPi = 3.14159265358979323846;
constexpr int kRayBins = 4;             // frequency bins per lane in one walk of a ray

// int_a^b x^3 / (e^x - 1) dx: composite 4-point Gauss-Legendre on panels of
// width <= 1/2 (at most 64); nothing beyond x = 300 (below 1e-120 of the peak)
__device__ double planck_x_integral(double a, double b) {
    const double gx0 = 0.33998104358485626, gx1 = 0.86113631159405258;
    const double gw0 = 0.65214515486254614, gw1 = 0.34785484513745386;
    if (!(b > a) || a > 300.0) return 0.0;
    const double w = b - a;
    int np = (int)ceil(w * 2.0);
    np = np < 1 ? 1 : (np > 64 ? 64 : np);
    const double h = w / np;
    double s = 0.0;
    for (int p = 0; p < np; ++p) {
        const double c = a + (p + 0.5) * h, r = 0.5 * h;
        const double x0 = c - r * gx1, x1 = c - r * gx0, x2 = c + r * gx0, x3 = c + r * gx1;
        s += gw1 * (x0 * x0 * x0 / expm1(x0) + x3 * x3 * x3 / expm1(x3)) +
             gw0 * (x1 * x1 * x1 / expm1(x1) + x2 * x2 * x2 / expm1(x2));
    }
    return 0.5 * h * s;
}

// image axes of the observer direction o, as for the peeled images
__device__ void image_axes(double o0, double o1, double o2, double* ex, double* ey) {
    double a = -o1, b = o0;
    const double en = sqrt(a * a + b * b);
    if (en < 1e-12) {
        a = 1.0;
        b = 0.0;
    } else {
        a /= en;
        b /= en;
    }
    ex[0] = a;
    ex[1] = b;
    ex[2] = 0.0;
    ey[0] = -o2 * b;
    ey[1] = o2 * a;
    ey[2] = o0 * b - o1 * a;
}

// A ray walk from x along d: current cell, ray parameter of the next wall per
// axis and its increment.  The start cell of a point on a wall is the cell the
// ray enters.
struct RayWalk {
    int c[3], step[3];
    double tn[3], dt[3];
    double t;
};

__device__ void walk_start(const RayParams& R, const double* x, const double* d, bool clamp, RayWalk& w) {
    for (int a = 0; a < 3; ++a) {
        const double f = (x[a] - R.lo[a]) / R.dx[a];
        const double fl = floor(f);
        int c = (int)fl;
        if (f == fl && d[a] < 0.0) c -= 1;
        if (clamp) c = c < 0 ? 0 : (c >= R.n[a] ? R.n[a] - 1 : c);
        w.c[a] = c;
        if (d[a] > 0.0) {
            w.step[a] = 1;
            w.tn[a] = (R.lo[a] + (c + 1) * R.dx[a] - x[a]) / d[a];
            w.dt[a] = R.dx[a] / d[a];
        } else if (d[a] < 0.0) {
            w.step[a] = -1;
            w.tn[a] = (R.lo[a] + c * R.dx[a] - x[a]) / d[a];
            w.dt[a] = -R.dx[a] / d[a];
        } else {
            w.step[a] = 0;
            w.tn[a] = INFINITY;
            w.dt[a] = INFINITY;
        }
    }
    w.t = 0.0;
}

__device__ __forceinline__ bool walk_inside(const RayParams& R, const RayWalk& w) {
    return (unsigned)w.c[0] < (unsigned)R.n[0] && (unsigned)w.c[1] < (unsigned)R.n[1] &&
           (unsigned)w.c[2] < (unsigned)R.n[2];
}

// chord through the current cell; moves to the next cell
__device__ __forceinline__ double walk_step(RayWalk& w, int64_t& j, const RayParams& R) {
    int ax = 0;
    if (w.tn[1] < w.tn[ax]) ax = 1;
    if (w.tn[2] < w.tn[ax]) ax = 2;
    const double l = fmax(w.tn[ax] - w.t, 0.0);
    j = w.c[0] + (int64_t)R.n[0] * (w.c[1] + (int64_t)R.n[1] * w.c[2]);
    w.t = fmax(w.tn[ax], w.t);
    w.tn[ax] += w.dt[ax];
    w.c[ax] += w.step[ax];
    return l;
}

__global__ void __launch_bounds__(256) k_raytrace_dust(RayParams R) {
    const int64_t npx2 = (int64_t)R.npix * R.npix;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int lane = threadIdx.x % kWave;
    if (wave >= (int64_t)R.n_obs * npx2) return;  // whole waves
    const int obs = (int)(wave / npx2);
    const int64_t pix = wave - obs * npx2;
    const int iy = (int)(pix / R.npix), ix = (int)(pix - (int64_t)iy * R.npix);
    const double* o = R.dirs + 3 * obs;
    double ex[3], ey[3];
    image_axes(o[0], o[1], o[2], ex, ey);
    const double wpix = 2.0 * R.hw / R.npix;
    const double X = -R.hw + (ix + 0.5) * wpix, Y = -R.hw + (iy + 0.5) * wpix;
    double q[3];
    for (int a = 0; a < 3; ++a) q[a] = 0.5 * (R.lo[a] + R.hi[a]) + X * ex[a] + Y * ey[a];
    // the line q + s o meets the grid box for s in [s0, s1]
    double s0 = -INFINITY, s1 = INFINITY;
    bool miss = false;
    for (int a = 0; a < 3; ++a) {
        if (o[a] != 0.0) {
            double u = (R.lo[a] - q[a]) / o[a], v = (R.hi[a] - q[a]) / o[a];
            if (u > v) {
                const double t = u;
                u = v;
                v = t;
            }
            s0 = fmax(s0, u);
            s1 = fmin(s1, v);
        } else if (q[a] < R.lo[a] || q[a] >= R.hi[a]) {
            miss = true;
        }
    }
    double* out = R.cube + wave * R.nnu;
    const double apix = wpix * wpix;
    if (miss || !(s1 > s0)) {
        for (int k = lane; k < R.nnu; k += kWave) out[k] = 0.0;
        return;
    }
    double x0[3], d[3];
    for (int a = 0; a < 3; ++a) {
        x0[a] = q[a] + s1 * o[a];
        d[a] = -o[a];
    }
    RayWalk w0;
    walk_start(R, x0, d, true, w0);
    // a lane holds bins k = lane + 64 i (i < kRayBins) through one walk of
    // the ray; more bins take further walks.  The attenuation in front is
    // carried as a product: one expm1 per bin and cell gives both 1 - e^-dtau
    // and the factor e^-dtau.
    for (int kb = 0; kb < R.nnu; kb += kWave * kRayBins) {
        double chi[kRayBins], sk[kRayBins], xlo[kRayBins], xhi[kRayBins], I[kRayBins], att[kRayBins];
#pragma unroll
        for (int i = 0; i < kRayBins; ++i) {
            const int k = kb + lane + kWave * i;
            const bool act = k < R.nnu;
            chi[i] = act ? R.chi[k] : 0.0;
            sk[i] = act ? R.kap[k] / R.chi[k] : 0.0;  // S = (kappa / chi) B
            xlo[i] = act ? kH * R.nu[k] : 0.0;        // h nu, divided by kT per cell
            xhi[i] = act ? kH * R.nu[k + 1] : 0.0;
            I[i] = 0.0;
            att[i] = 1.0;
        }
        RayWalk w = w0;
        while (walk_inside(R, w)) {
            int64_t j;
            const double l = walk_step(w, j, R);
            const double r = R.rho[j];
            if (!(r > 0.0)) continue;
            const double T = R.T[j];
            // B_k(T) from the table: cubic Hermite interpolation of ln B in ln T
            // on rows dlnT apart (the same row and weights for every bin of the
            // cell); quadrature outside the table's range
            const bool tab = T >= kTLo && T <= kTHi;
            int row = 0;
            double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
            if (tab) {
                const double u = (log(T) - log(kTLo)) / R.dlnT;
                row = (int)u;
                row = row > kRayTRows - 2 ? kRayTRows - 2 : row;
                const double f = u - row, f2 = f * f, f3 = f2 * f;
                w0 = 2.0 * f3 - 3.0 * f2 + 1.0;           // value at row
                w1 = (f3 - 2.0 * f2 + f) * R.dlnT;         // slope at row
                w2 = -2.0 * f3 + 3.0 * f2;                 // value at row + 1
                w3 = (f3 - f2) * R.dlnT;                   // slope at row + 1
            }
            const double kT = kKB * T;
            const double pref = T > 0.0 ? 2.0 * kT * kT * kT * kT / (kH * kH * kH * kC * kC) : 0.0;
            const double ikT = T > 0.0 ? 1.0 / kT : 0.0;
#pragma unroll
            for (int i = 0; i < kRayBins; ++i) {
                const int k = kb + lane + kWave * i;
                const double em = expm1(-r * chi[i] * l);  // e^-dtau - 1
                double S = 0.0;
                if (tab) {
                    if (k < R.nnu) {
                        const double2 e0 = R.btab[(size_t)row * R.nnu + k];
                        const double2 e1 = R.btab[(size_t)(row + 1) * R.nnu + k];
                        S = sk[i] * exp(w0 * e0.x + w1 * e0.y + w2 * e1.x + w3 * e1.y);
                    }
                } else if (T > 0.0) {
                    S = sk[i] * pref * planck_x_integral(xlo[i] * ikT, xhi[i] * ikT);
                }
                I[i] += att[i] * S * -em;
                att[i] *= 1.0 + em;
            }
        }
#pragma unroll
        for (int i = 0; i < kRayBins; ++i) {
            const int k = kb + lane + kWave * i;
            if (k < R.nnu) out[k] = I[i] * apix;
        }
    }
}

// sed[o][1][k] = sum over the pixels of cube[o][.][.][k]
__global__ void __launch_bounds__(256) k_raytrace_sum(RayParams R, int slices) {
    const int obs = blockIdx.x / slices, sl = blockIdx.x % slices;
    const int64_t npx2 = (int64_t)R.npix * R.npix;
    const int64_t p0 = npx2 * sl / slices, p1 = npx2 * (sl + 1) / slices;
    for (int k = threadIdx.x; k < R.nnu; k += blockDim.x) {
        double s = 0.0;
        for (int64_t p = p0; p < p1; ++p) s += R.cube[((int64_t)obs * npx2 + p) * R.nnu + k];
        if (s != 0.0) unsafeAtomicAdd(R.sed + ((size_t)obs * 2 + 1) * R.nnu + k, s);
    }
}

// one wave per (observer, source): L_k / (4 pi) exp(-tau_k) into sed[o][0][k]
// and into the pixel the source projects into
__global__ void __launch_bounds__(256) k_raytrace_sources(RayParams R) {
    const int wave = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
    const int lane = threadIdx.x % kWave;
    if (wave >= R.n_obs * R.nsrc) return;
    const int obs = wave / R.nsrc, src = wave % R.nsrc;
    const double* o = R.dirs + 3 * obs;
    const double* p = R.spos + 3 * src;
    double ex[3], ey[3], pc[3];
    image_axes(o[0], o[1], o[2], ex, ey);
    for (int a = 0; a < 3; ++a) pc[a] = p[a] - 0.5 * (R.lo[a] + R.hi[a]);
    const double X = pc[0] * ex[0] + pc[1] * ex[1] + pc[2] * ex[2];
    const double Y = pc[0] * ey[0] + pc[1] * ey[1] + pc[2] * ey[2];
    const double fx = floor((X + R.hw) / (2.0 * R.hw) * R.npix);
    const double fy = floor((Y + R.hw) / (2.0 * R.hw) * R.npix);
    const bool in_img = fx >= 0.0 && fy >= 0.0 && fx < R.npix && fy < R.npix;
    RayWalk w0;
    walk_start(R, p, o, false, w0);
    for (int kb = 0; kb < R.nnu; kb += kWave) {
        const int k = kb + lane;
        const bool act = k < R.nnu;
        const double chi = act ? R.chi[k] : 0.0;
        double tau = 0.0;
        RayWalk w = w0;
        while (walk_inside(R, w)) {
            int64_t j;
            const double l = walk_step(w, j, R);
            tau += R.rho[j] * chi * l;
        }
        if (act) {
            const double v = R.lsrc[(size_t)src * R.nnu + k] / (4.0 * kPi) * exp(-tau);
            unsafeAtomicAdd(R.sed + ((size_t)obs * 2) * R.nnu + k, v);
            if (in_img)
                unsafeAtomicAdd(R.cube + ((((size_t)obs * R.npix + (size_t)fy) * R.npix + (size_t)fx) *
                                              R.nnu + k), v);
        }
    }
}

}  // namespace

hipError_t launch_raytrace(const RayParams& R, hipStream_t st) {
    const int64_t waves = (int64_t)R.n_obs * R.npix * R.npix;
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_raytrace_dust, dim3((unsigned)blocks), dim3(256), 0, st, R);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int slices = 64;
    hipLaunchKernelGGL(k_raytrace_sum, dim3(R.n_obs * slices), dim3(256), 0, st, R, slices);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (R.nsrc > 0) {
        const int sb = (R.n_obs * R.nsrc + 3) / 4;
        hipLaunchKernelGGL(k_raytrace_sources, dim3(sb), dim3(256), 0, st, R);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace mcrt
