// mcrt_cells.hip -- per-cell kernels of a Lucy iteration (Robitaille 2011,
// Sec. 2.3 Eqs. 2-3, Sec. 2.4 Eqs. 4-6), all FP64 and streaming:
//   k_rows       temperature -> emissivity row position for the next pass
//   k_update     Adot from the path-length tally, T from the LTE balance,
//                per-cell convergence ratios into scratch buffers
//   k_hist/k_pick  radix selection of a nearest-rank percentile
#include <math.h>

#include "mcrt_internal.h"

namespace mcrt {

// Row position p = (kRows-1) ln(T/1K) / ln(1e4), clamped to [0, kRows-1]; the
// emitting row is floor(p) or floor(p)+1 with weight p - floor(p).
template <typename R>
__global__ void k_rows(int64_t ncell, const double* __restrict__ T, const double* __restrict__ rho,
                       R* __restrict__ rowpos, unsigned long long* __restrict__ n_clamped) {
    const double scale = (double)(kRows - 1) / log(kTHi / kTLo);
    unsigned long long c = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double t = T[j];
        double p = scale * log(t / kTLo);
        if ((t < kTLo || t > kTHi) && rho[j] > 0.0) ++c;
        p = fmin((double)(kRows - 1), fmax(0.0, p));
        rowpos[j] = (R)p;
    }
    // wave reduction, one atomic per wave
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0 && c) atomicAdd(n_clamped, c);
}

// T from ln Adot by the table of ln Adot(ln T) (rows uniform in ln T from
// ln 1 K): bracket by bisection, then invert the cubic Hermite interpolant on
// the bracket with Newton steps.  Returns T and dlnAdot/dlnT.
__device__ __forceinline__ double solve_T(const double* __restrict__ lnA,
                                          const double* __restrict__ slope, double dy, double la,
                                          double* dlnA_dlnT, int* clamped) {
    *clamped = 0;
    if (la <= lnA[0]) {
        *clamped = la < lnA[0];
        *dlnA_dlnT = slope[0];
        return kTLo;
    }
    if (la >= lnA[kTSolveRows - 1]) {
        *clamped = la > lnA[kTSolveRows - 1];
        *dlnA_dlnT = slope[kTSolveRows - 1];
        return kTHi;
    }
    int lo = 0, hi = kTSolveRows - 1;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (lnA[mid] <= la) lo = mid;
        else hi = mid;
    }
    const double f0 = lnA[lo], f1 = lnA[hi];
    const double m0 = slope[lo] * dy, m1 = slope[hi] * dy;
    double t = (la - f0) / (f1 - f0);
    double der = 1.0;
    for (int it = 0; it < 4; ++it) {
        const double t2 = t * t, t3 = t2 * t;
        const double h00 = 2 * t3 - 3 * t2 + 1, h10 = t3 - 2 * t2 + t;
        const double h01 = -2 * t3 + 3 * t2, h11 = t3 - t2;
        const double f = h00 * f0 + h10 * m0 + h01 * f1 + h11 * m1;
        const double d00 = 6 * t2 - 6 * t, d10 = 3 * t2 - 4 * t + 1;
        const double d01 = -6 * t2 + 6 * t, d11 = 3 * t2 - 2 * t;
        der = d00 * f0 + d10 * m0 + d01 * f1 + d11 * m1;
        t -= (f - la) / der;
        t = fmin(1.0, fmax(0.0, t));
    }
    *dlnA_dlnT = der / dy;
    return exp((lo + t) * dy);
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Adot by Eq. 2 (Delta t = 1 s), T by Eq. 3 over the bins, and the per-cell
// inputs of the convergence statistics:
//   R_j = delta(Adot^{i-1}, Adot^i) for dust cells sampled in both iterations
//   r_j = |T^i - T^{i-1}| / T^{i-1} over the mask (dust, sampled now, previous
//         T valid, and -- with the noise estimate -- sigma_dT/T below a limit)
// Cells outside a set get +inf so that a selection over the set ignores them.
// index of x-fastest cell j in the 4x4x4 brick layout of the transport arrays
__device__ __forceinline__ int64_t brick_index(int64_t j, int nx, int ny, int bx, int bxy) {
    const int64_t nxy = (int64_t)nx * ny;
    const int c2 = (int)(j / nxy);
    const int64_t r = j - (int64_t)c2 * nxy;
    const int c1 = (int)(r / nx);
    const int c0 = (int)(r - (int64_t)c1 * nx);
    return ((int64_t)((c2 >> 2) * bxy + (c1 >> 2) * bx + (c0 >> 2)) << 6) | ((c2 & 3) << 4) |
           ((c1 & 3) << 2) | (c0 & 3);
}

__global__ void k_update(CellParams P) {
    unsigned long long n_r = 0, n_mask = 0, n_uns = 0, n_cl = 0;
    double rmax = 0.0;
    const double INF = __builtin_inf();
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t jt = P.brick ? brick_index(j, P.n[0], P.n[1], P.bx, P.bxy) : j;
        double tally = 0.0;
        for (int c = 0; c < P.acc_copies; ++c) tally += P.acc[jt + (size_t)c * P.acc_stride];
        const double a = P.eps_over_vol * tally;
        const double Tp = P.T[j];
        const double sp = P.sig_rel[j];
        const unsigned char vp = P.valid[j];
        const double ap = P.adot[j];
        const double rho = P.rho[j];
        P.T_prev[j] = Tp;
        P.sig_rel_prev[j] = sp;
        P.valid_prev[j] = vp;
        P.adot_prev[j] = ap;
        P.adot[j] = a;
        double sig = 0.0;
        if (P.acc2) {
            sig = P.eps_over_vol * sqrt(P.acc2[jt]);
            P.adot_sig[j] = sig;
        }
        double T, srel = 0.0;
        unsigned char v;
        if (a > 0.0) {
            double dl;
            int cl;
            T = solve_T(P.lnA, P.slope, P.dy, log(a), &dl, &cl);
            n_cl += cl;
            v = 1;
            if (P.want_noise) srel = (sig / a) / dl;
        } else {
            T = kTFloor;
            v = 0;
            if (rho > 0.0) ++n_uns;
        }
        P.T[j] = T;
        P.sig_rel[j] = srel;
        P.valid[j] = v;
        double R = INF;
        if (P.have_prev && rho > 0.0 && ap > 0.0 && a > 0.0) {
            R = ap > a ? ap / a : a / ap;
            ++n_r;
        }
        P.Rbuf[j] = R;
        double r = INF;
        if (rho > 0.0 && a > 0.0 && vp) {
            bool ok = true;
            if (P.want_noise) ok = sqrt(srel * srel + sp * sp) <= P.noise_thres;
            if (ok) {
                r = fabs(T - Tp) / Tp;
                rmax = fmax(rmax, r);
                ++n_mask;
            }
        }
        P.rbuf[j] = r;
    }
    n_r = wave_sum(n_r);
    n_mask = wave_sum(n_mask);
    n_uns = wave_sum(n_uns);
    n_cl = wave_sum(n_cl);
    rmax = wave_max(rmax);
    if (__lane_id() == 0) {
        if (n_r) atomicAdd(P.stats + 0, n_r);
        if (n_mask) atomicAdd(P.stats + 1, n_mask);
        if (n_uns) atomicAdd(P.stats + 2, n_uns);
        if (n_cl) atomicAdd(P.stats + 3, n_cl);
        // non-negative doubles order like their bit patterns
        atomicMax(P.stats + 4, (unsigned long long)__double_as_longlong(rmax));
    }
}

// ---------------------------------------------------------------------------
// Nearest-rank percentile by radix selection over the bit patterns of
// non-negative doubles (8 passes of 8 bits).  sel[0] = prefix found so far,
// sel[1] = rank still to find inside the prefix (0-based), sel[2] = pass.
// ---------------------------------------------------------------------------
__global__ void k_hist(int64_t n, const double* __restrict__ v,
                       const unsigned long long* __restrict__ sel, unsigned int* __restrict__ hist) {
    __shared__ unsigned int h[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) h[i] = 0;
    __syncthreads();
    const unsigned long long prefix = sel[0];
    const int pass = (int)sel[2];
    const int shift = 56 - 8 * pass;
    const unsigned long long mask_hi = pass == 0 ? 0ull : (~0ull << (64 - 8 * pass));
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long b = (unsigned long long)__double_as_longlong(v[j]);
        if ((b & mask_hi) == prefix) atomicAdd(&h[(b >> shift) & 255ull], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x)
        if (h[i]) atomicAdd(hist + i, h[i]);
}

__global__ void k_pick(unsigned long long* sel, unsigned int* hist) {
    if (threadIdx.x == 0) {
        const int pass = (int)sel[2];
        const int shift = 56 - 8 * pass;
        unsigned long long rank = sel[1];
        unsigned long long acc = 0;
        int d = 0;
        for (; d < 256; ++d) {
            if (acc + hist[d] > rank) break;
            acc += hist[d];
        }
        if (d > 255) d = 255;
        sel[0] |= (unsigned long long)d << shift;
        sel[1] = rank - acc;
        sel[2] = pass + 1;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 256; i += blockDim.x) hist[i] = 0;
}

hipError_t launch_rows64(int64_t ncell, const double* T, const double* rho, double* rowpos,
                         unsigned long long* nclamp, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_rows<double>, dim3(blocks), dim3(256), 0, st, ncell, T, rho, rowpos, nclamp);
    return hipGetLastError();
}
hipError_t launch_rows32(int64_t ncell, const double* T, const double* rho, float* rowpos,
                         unsigned long long* nclamp, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_rows<float>, dim3(blocks), dim3(256), 0, st, ncell, T, rho, rowpos, nclamp);
    return hipGetLastError();
}
hipError_t launch_update(const CellParams& P, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_update, dim3(blocks), dim3(256), 0, st, P);
    return hipGetLastError();
}
// Select the rank-th smallest (0-based) value of v; the result's bits end in sel[0].
hipError_t launch_select(int64_t n, const double* v, unsigned long long* sel, unsigned int* hist,
                         int blocks, hipStream_t st) {
    for (int pass = 0; pass < 8; ++pass) {
        hipLaunchKernelGGL(k_hist, dim3(blocks), dim3(256), 0, st, n, v, sel, hist);
        hipLaunchKernelGGL(k_pick, dim3(1), dim3(256), 0, st, sel, hist);
    }
    return hipGetLastError();
}

}  // namespace mcrt

// ---------------------------------------------------------------------------
// small element-wise helpers (conversions, fills, validation of device input)
// ---------------------------------------------------------------------------
namespace mcrt {

__global__ void k_to_f32(int64_t n, const double* __restrict__ in, float* __restrict__ out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        out[j] = (float)in[j];
}
__global__ void k_to_f64(int64_t n, const float* __restrict__ in, double* __restrict__ out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        out[j] = (double)in[j];
}
__global__ void k_fill_u8(int64_t n, unsigned char* p, unsigned char v) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}
__global__ void k_add_u32(int64_t n, uint32_t* p, uint32_t v) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        p[j] += v;
}
hipError_t launch_add_u32(int64_t n, uint32_t* p, uint32_t v, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_add_u32, dim3(blocks), dim3(256), 0, st, n, p, v);
    return hipGetLastError();
}
__global__ void k_fill_u64(int64_t n, unsigned long long* p, unsigned long long v) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}
hipError_t launch_fill_u64(int64_t n, unsigned long long* p, unsigned long long v, int blocks,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u64, dim3(blocks), dim3(256), 0, st, n, p, v);
    return hipGetLastError();
}
__global__ void k_fill_f64(int64_t n, double* p, double v) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        p[j] = v;
}
// counts entries that are not finite or not above `lo` (strict) / below 0 (lo < 0)
__global__ void k_count_bad(int64_t n, const double* __restrict__ v, int strict_positive,
                            unsigned long long* bad) {
    unsigned long long c = 0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double x = v[j];
        const bool ok = isfinite(x) && (strict_positive ? x > 0.0 : x >= 0.0);
        c += ok ? 0 : 1;
    }
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
    if (__lane_id() == 0 && c) atomicAdd(bad, c);
}

// x-fastest -> 4x4x4 bricks (pad cells of partial bricks keep their zero)
template <typename T>
__global__ void k_to_bricks(int64_t n, int nx, int ny, int bx, int bxy, const T* __restrict__ in,
                            T* __restrict__ out) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        out[brick_index(j, nx, ny, bx, bxy)] = in[j];
}
hipError_t launch_to_bricks_f32(int64_t n, int nx, int ny, int bx, int bxy, const float* in,
                                float* out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bricks<float>, dim3(blocks), dim3(256), 0, st, n, nx, ny, bx, bxy, in, out);
    return hipGetLastError();
}
hipError_t launch_to_bricks_f64(int64_t n, int nx, int ny, int bx, int bxy, const double* in,
                                double* out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_to_bricks<double>, dim3(blocks), dim3(256), 0, st, n, nx, ny, bx, bxy, in, out);
    return hipGetLastError();
}

hipError_t launch_to_f32(int64_t n, const double* in, float* out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, st, n, in, out);
    return hipGetLastError();
}
hipError_t launch_to_f64(int64_t n, const float* in, double* out, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_to_f64, dim3(blocks), dim3(256), 0, st, n, in, out);
    return hipGetLastError();
}
hipError_t launch_fill_u8(int64_t n, unsigned char* p, unsigned char v, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_u8, dim3(blocks), dim3(256), 0, st, n, p, v);
    return hipGetLastError();
}
hipError_t launch_fill_f64(int64_t n, double* p, double v, int blocks, hipStream_t st) {
    hipLaunchKernelGGL(k_fill_f64, dim3(blocks), dim3(256), 0, st, n, p, v);
    return hipGetLastError();
}
hipError_t launch_check_T(int64_t n, const double* T, unsigned long long* bad, int blocks,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_count_bad, dim3(blocks), dim3(256), 0, st, n, T, 1, bad);
    return hipGetLastError();
}
hipError_t launch_check_rho(int64_t n, const double* rho, unsigned long long* bad, int blocks,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_count_bad, dim3(blocks), dim3(256), 0, st, n, rho, 0, bad);
    return hipGetLastError();
}

}  // namespace mcrt
