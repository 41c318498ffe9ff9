// mcrt_pda.hip -- partial diffusion approximation (Appendix A) on the GPU.
//
// Cells that the packets sample poorly (zero absorption, or a relative error
// of the absorption estimate above a threshold) take their temperature from
// div(D grad T^4) = 0, D = 1 / (3 rho chi_R), with the sampled cells around
// them as boundary values.  The Cartesian form of the appendix's discrete
// equation couples a cell c to a face neighbour n along axis a with the
// conductance g = 1 / (dx_a^2 (rho_c chi_R,c + rho_n chi_R,n)); empty cells
// and the outside of the grid carry no flux.  The linear system over the PDA
// cells connected to a sampled cell is symmetric positive definite and is
// solved matrix-free by conjugate gradients with a Jacobi preconditioner: one
// 7-point stencil per iteration, coalesced over x-fastest cells, with FP64
// block reductions.  Groups of PDA cells without a sampled neighbour are found
// by flag propagation and left as they are.
#include <math.h>

#include "mcrt_internal.h"

namespace mcrt {

namespace {

constexpr int kPdaBlock = 256;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_down(v, o);
    const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
    if (l == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int i = 0; i < (int)blockDim.x / kWave; ++i) s += sh[i];
    __syncthreads();
    return s;  // valid in thread 0
}

__device__ __forceinline__ void neighbour(const PdaParams& P, int64_t j, int q, int64_t& nb, double& dx) {
    const int nx = P.n[0], ny = P.n[1], nz = P.n[2];
    const int x = (int)(j % nx), y = (int)((j / nx) % ny), z = (int)(j / ((int64_t)nx * ny));
    const int ax = q >> 1, s = (q & 1) ? 1 : -1;
    const int c = ax == 0 ? x : (ax == 1 ? y : z);
    const int size = P.n[ax];
    dx = P.dx[ax];
    if (c + s < 0 || c + s >= size) {
        nb = -1;
        return;
    }
    nb = j + s * (ax == 0 ? (int64_t)1 : (ax == 1 ? (int64_t)nx : (int64_t)nx * ny));
}

// Rosseland-mean chi at T: cubic Hermite in ln T of the kMrwRows table
// (kappa_P, d kappa_P, chi_R, d chi_R per row)
__device__ __forceinline__ double chi_rosseland(const double* tab, double T) {
    const double lo = log(kTLo), h = (log(kTHi) - lo) / (kMrwRows - 1);
    double p = (log(T) - lo) / h;
    p = fmin(fmax(p, 0.0), (double)(kMrwRows - 1));
    int i = (int)p;
    i = i > kMrwRows - 2 ? kMrwRows - 2 : i;
    const double t = p - i, t2 = t * t, t3 = t2 * t;
    const double* a = tab + 4 * (size_t)i;
    const double* b = a + 4;
    return (2 * t3 - 3 * t2 + 1) * a[2] + (t3 - 2 * t2 + t) * h * a[3] + (-2 * t3 + 3 * t2) * b[2] +
           (t3 - t2) * h * b[3];
}

// flags (select): 1 PDA cell (not yet connected); a = rho chi_R(T) on dust
// cells (at every Picard pass)
__global__ void k_pda_coefficients(PdaParams P, int select) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double r = P.rho[j];
        if (select) {
            unsigned char f = 0;
            if (r > 0.0) {
                const double A = P.adot[j];
                if (A <= 0.0 || (P.adot_sig && P.adot_sig[j] > P.noise * A)) f = 1;
            }
            P.flag[j] = f;
            const unsigned long long w = __ballot(f != 0);
            if (__lane_id() == 0 && w) atomicAdd(P.count, (unsigned)__popcll(w));
        }
        P.a[j] = r > 0.0 ? r * chi_rosseland(P.mrw_tab, P.T[j]) : 0.0;
    }
}

// one round of connection: a PDA cell next to a sampled dust cell or to a
// connected PDA cell becomes connected; counts changes
__global__ void k_pda_connect(PdaParams P) {
    unsigned changed = 0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (P.flag[j] != 1) continue;
        for (int q = 0; q < 6; ++q) {
            int64_t nb;
            double dx;
            neighbour(P, j, q, nb, dx);
            if (nb < 0 || !(P.rho[nb] > 0.0)) continue;
            const unsigned char fn = P.flag[nb];
            if (fn == 0 || fn == 2) {
                P.flag[j] = 2;
                ++changed;
                break;
            }
        }
    }
    if (changed) atomicAdd(P.count, changed);
}

// conductance sum (diagonal), boundary term b, initial x = T^4 and the first
// residual r = b - A x, z = r / diag, p = z; rz and bb reductions
__global__ void __launch_bounds__(kPdaBlock) k_pda_init(PdaParams P) {
    __shared__ double sh[2][kPdaBlock / kWave];
    double rz = 0.0, bb = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (P.flag[j] != 2) {
            P.x[j] = P.r[j] = P.z[j] = P.p[j] = 0.0;
            continue;
        }
        const double Tj = P.T[j], u = Tj * Tj * Tj * Tj;
        double d = 0.0, b = 0.0, Ax = 0.0;
        for (int q = 0; q < 6; ++q) {
            int64_t nb;
            double dx;
            neighbour(P, j, q, nb, dx);
            if (nb < 0 || !(P.rho[nb] > 0.0)) continue;
            const double g = 1.0 / (dx * dx * (P.a[j] + P.a[nb]));
            d += g;
            const double Tn = P.T[nb];
            if (P.flag[nb] == 2) Ax -= g * Tn * Tn * Tn * Tn;
            else b += g * Tn * Tn * Tn * Tn;
        }
        Ax += d * u;
        P.diag[j] = d;
        P.b[j] = b;
        P.x[j] = u;
        const double r = b - Ax;
        P.r[j] = r;
        P.z[j] = r / d;
        P.p[j] = r / d;
        rz += r * r / d;
        bb += b * b;
    }
    rz = block_sum(rz, sh[0]);
    bb = block_sum(bb, sh[1]);
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(P.red + 0, rz);
        unsafeAtomicAdd(P.red + 4, bb);
    }
}

// q = A p and p.q
__global__ void __launch_bounds__(kPdaBlock) k_pda_apply(PdaParams P) {
    __shared__ double sh[kPdaBlock / kWave];
    double pq = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (P.flag[j] != 2) continue;
        double s = P.diag[j] * P.p[j];
        for (int q = 0; q < 6; ++q) {
            int64_t nb;
            double dx;
            neighbour(P, j, q, nb, dx);
            if (nb < 0 || P.flag[nb] != 2) continue;
            s -= P.p[nb] / (dx * dx * (P.a[j] + P.a[nb]));
        }
        P.q[j] = s;
        pq += P.p[j] * s;
    }
    pq = block_sum(pq, sh);
    if (threadIdx.x == 0) unsafeAtomicAdd(P.red + 1, pq);
}

// alpha = rz / pq; x += alpha p; r -= alpha q; z = r / diag; new rz and rr
__global__ void __launch_bounds__(kPdaBlock) k_pda_step(PdaParams P) {
    __shared__ double sh[2][kPdaBlock / kWave];
    const double alpha = P.red[0] / P.red[1];
    double rz = 0.0, rr = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (P.flag[j] != 2) continue;
        P.x[j] += alpha * P.p[j];
        const double r = P.r[j] - alpha * P.q[j];
        P.r[j] = r;
        const double z = r / P.diag[j];
        P.z[j] = z;
        rz += r * z;
        rr += r * r;
    }
    rz = block_sum(rz, sh[0]);
    rr = block_sum(rr, sh[1]);
    if (threadIdx.x == 0) {
        unsafeAtomicAdd(P.red + 2, rz);
        unsafeAtomicAdd(P.red + 3, rr);
    }
}

// p = z + (rz_new / rz) p
__global__ void k_pda_direction(PdaParams P) {
    const double beta = P.red[2] / P.red[0];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x)
        if (P.flag[j] == 2) P.p[j] = P.z[j] + beta * P.p[j];
}

// rz <- rz_new, and the accumulators of the next iteration cleared
__global__ void k_pda_shift(PdaParams P) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        P.red[0] = P.red[2];
        P.red[1] = 0.0;
        P.red[2] = 0.0;
        P.red[3] = 0.0;
    }
}

// T = x^(1/4) and Adot(T) from the ln Adot(ln T) table (cubic Hermite, rows
// uniform in ln T from ln 1 K) on the connected PDA cells
__global__ void k_pda_finish(PdaParams P) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < P.ncell;
         j += (int64_t)gridDim.x * blockDim.x) {
        if (P.flag[j] != 2) continue;
        double T = sqrt(sqrt(fmax(P.x[j], 0.0)));
        T = fmin(fmax(T, kTLo), kTHi);
        double pos = log(T) / P.dy;
        pos = fmin(fmax(pos, 0.0), (double)(kTSolveRows - 1));
        int i = (int)pos;
        i = i > kTSolveRows - 2 ? kTSolveRows - 2 : i;
        const double t = pos - i, t2 = t * t, t3 = t2 * t;
        const double la = (2 * t3 - 3 * t2 + 1) * P.lnA[i] + (t3 - 2 * t2 + t) * P.slope[i] * P.dy +
                          (-2 * t3 + 3 * t2) * P.lnA[i + 1] + (t3 - t2) * P.slope[i + 1] * P.dy;
        P.T[j] = T;
        P.adot_out[j] = exp(la);
        P.valid[j] = 1;
    }
}

int grid_of(int64_t n) {
    const int64_t b = (n + kPdaBlock - 1) / kPdaBlock;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

}  // namespace

hipError_t launch_pda_coefficients(const PdaParams& P, int select, hipStream_t st) {
    hipLaunchKernelGGL(k_pda_coefficients, dim3(grid_of(P.ncell)), dim3(kPdaBlock), 0, st, P, select);
    return hipGetLastError();
}

hipError_t launch_pda_connect(const PdaParams& P, hipStream_t st) {
    hipLaunchKernelGGL(k_pda_connect, dim3(grid_of(P.ncell)), dim3(kPdaBlock), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_pda_init(const PdaParams& P, hipStream_t st) {
    hipLaunchKernelGGL(k_pda_init, dim3(grid_of(P.ncell)), dim3(kPdaBlock), 0, st, P);
    return hipGetLastError();
}

// one conjugate-gradient iteration (the caller reads red[3] = r.r afterwards)
hipError_t launch_pda_iteration(const PdaParams& P, hipStream_t st) {
    const int g = grid_of(P.ncell);
    hipLaunchKernelGGL(k_pda_apply, dim3(g), dim3(kPdaBlock), 0, st, P);
    hipLaunchKernelGGL(k_pda_step, dim3(g), dim3(kPdaBlock), 0, st, P);
    hipLaunchKernelGGL(k_pda_direction, dim3(g), dim3(kPdaBlock), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_pda_shift(const PdaParams& P, hipStream_t st) {
    hipLaunchKernelGGL(k_pda_shift, dim3(1), dim3(64), 0, st, P);
    return hipGetLastError();
}

hipError_t launch_pda_finish(const PdaParams& P, hipStream_t st) {
    hipLaunchKernelGGL(k_pda_finish, dim3(grid_of(P.ncell)), dim3(kPdaBlock), 0, st, P);
    return hipGetLastError();
}

}  // namespace mcrt
