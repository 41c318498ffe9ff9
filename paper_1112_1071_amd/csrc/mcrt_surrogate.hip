// mcrt_surrogate.hip -- gfx950 kernels of the learned warm start: a 3-D
// convolutional encoder-decoder evaluated and trained with BF16 operands on
// the matrix cores (FP32 accumulation).  The 3x3x3 convolutions, which carry
// nearly all of the work, stage a brick of their input with its one-voxel
// halo in LDS and run on v_mfma_f32_16x16x32_bf16 (forward, backward data and
// weight gradients); the stride-2 down and up convolutions use a plain
// per-lane gather on v_mfma_f32_16x16x16_bf16.
//
// Tensors are channels-last (voxel-major, channel fastest) BF16.  Every
// convolution is an implicit GEMM: rows = voxels, columns = output channels,
// reduction = taps x input channels, in one of three geometries:
//   CONV3  3x3x3 taps, stride 1, zero padding 1
//   DOWN   2x2x2 taps, stride 2 (output grid half the input grid)
//   UP     transposed 2x2x2, stride 2: an output voxel 2u+p receives input
//          voxel u through tap p only, so each parity class p is a plain GEMM
// A second input tensor may follow the first along the channel axis (the
// skip concatenation of the decoder) without being copied.  The backward
// data pass reuses the same kernel: CONV3 with flipped taps, DOWN <-> UP,
// with the weights transposed; weight gradients are an MFMA reduction over
// voxels.  Channel counts are multiples of 16.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcrt {
namespace nn {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef short s16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// D += A B with A 16x32, B 32x16 (BF16), D 16x16 (FP32).  Lane l holds
// A[l % 16][8 (l / 16) + j] and B[8 (l / 16) + j][l % 16] for j = 0..7, and
// D[4 (l / 16) + i][l % 16] for i = 0..3.
__device__ __forceinline__ f32x4 mfma32(const uint4& a, const uint4& b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                   c, 0, 0, 0);
}

enum Mode : int { CONV3 = 0, DOWN = 1, UP = 2 };

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ uint16_t f2bf(float x) {
    __hip_bfloat16 b = __float2bfloat16(x);  // round to nearest even
    return *reinterpret_cast<uint16_t*>(&b);
}

struct ConvArgs {
    const uint16_t* in1;  // [N][Din^3][C1]
    const uint16_t* in2;  // [N][Din^3][C2] or null
    int C1, C2;
    const uint16_t* w;    // [taps][Cout][C1+C2]
    const float* bias;    // [Cout] or null
    int Cout;
    int N, Din, Dout;     // grid sides (cubic)
    int mode;
    // output: BF16 with LeakyReLU (forward) or FP32 accumulate (backward data),
    // channels [0, Csplit) to out (stride Csplit) and the rest to out2
    uint16_t* out_bf;
    float* out_f;
    float* out_f2;
    int Csplit;
    int act;              // apply LeakyReLU
    float slope;
    int accumulate;       // FP32 output: add to the existing value
};

// source voxel of GEMM row r (a voxel of the row grid) and tap t; -1 if padding.
// Rows: CONV3/DOWN -> output voxels (grid Dout); UP -> input voxels (grid Din).
// The row's decomposition runs in the index type I: 32-bit whenever the
// launch's rows and voxels fit (every network size here), 64-bit otherwise.
template <typename I>
__device__ __forceinline__ int64_t src_voxel(const ConvArgs& A, int64_t r, int t) {
    if (A.mode == UP) return r;
    const I Dg = (I)A.Dout;
    const I per = Dg * Dg * Dg;
    const I rr = (I)r;
    const I n = rr / per;
    I q = rr - n * per;
    const I z = q / (Dg * Dg);
    q -= z * Dg * Dg;
    const I y = q / Dg, x = q - y * Dg;
    int sz, sy, sx;
    if (A.mode == CONV3) {
        sz = (int)z + t / 9 - 1;
        sy = (int)y + (t / 3) % 3 - 1;
        sx = (int)x + t % 3 - 1;
        if ((unsigned)sz >= (unsigned)A.Din || (unsigned)sy >= (unsigned)A.Din ||
            (unsigned)sx >= (unsigned)A.Din)
            return -1;
    } else {
        sz = 2 * (int)z + (t >> 2);
        sy = 2 * (int)y + ((t >> 1) & 1);
        sx = 2 * (int)x + (t & 1);
    }
    const I Di = (I)A.Din;
    return (int64_t)(((n * Di + (I)sz) * Di + (I)sy) * Di + (I)sx);
}

// output voxel of GEMM row r (parity class p for UP)
template <typename I>
__device__ __forceinline__ int64_t dst_voxel(const ConvArgs& A, int64_t r, int p) {
    if (A.mode != UP) return r;
    const I Dg = (I)A.Din;
    const I per = Dg * Dg * Dg;
    const I rr = (I)r;
    const I n = rr / per;
    I q = rr - n * per;
    const I z = q / (Dg * Dg);
    q -= z * Dg * Dg;
    const I y = q / Dg, x = q - y * Dg;
    const I Do = (I)A.Dout;
    return (int64_t)(((n * Do + 2 * z + (I)(p >> 2)) * Do + 2 * y + (I)((p >> 1) & 1)) * Do + 2 * x +
                     (I)(p & 1));
}

// Implicit-GEMM convolution.  A workgroup of 4 waves covers 64 rows; each wave
// 16 rows x 64 output channels (4 MFMA tiles) of blockIdx.y's channel block.
template <typename I>
__global__ void __launch_bounds__(256) k_conv(ConvArgs A, int64_t rows) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
    const int co0 = blockIdx.y * 64;
    const int ntile = min(4, (A.Cout - co0) / 16);
    const int p = blockIdx.z;  // UP: parity class
    const int taps = A.mode == CONV3 ? 27 : 8;
    const int Cin = A.C1 + A.C2;
    const int m = lane & 15, kq = lane >> 4;  // A: row m, channels 4kq..4kq+3
    const int64_t row = r0 + m;
    const bool row_ok = row < rows;
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int t_lo = A.mode == UP ? p : 0, t_hi = A.mode == UP ? p + 1 : taps;
    for (int t = t_lo; t < t_hi; ++t) {
        const int64_t sv = row_ok ? src_voxel<I>(A, row, t) : -1;
        const uint16_t* wt = A.w + (size_t)t * A.Cout * Cin;
        for (int c0 = 0; c0 < Cin; c0 += 16) {
            bf16x4 a = {0, 0, 0, 0};
            if (sv >= 0) {
                const int c = c0 + 4 * kq;
                const uint16_t* src = c < A.C1 ? A.in1 + sv * A.C1 + c : A.in2 + sv * A.C2 + (c - A.C1);
                a = *reinterpret_cast<const bf16x4*>(src);
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
                if (tt < ntile) {
                    // B: k = channel c0+4kq+i, n = output channel co0+16tt+m
                    const uint16_t* wp = wt + (size_t)(co0 + 16 * tt + m) * Cin + c0 + 4 * kq;
                    const bf16x4 b = *reinterpret_cast<const bf16x4*>(wp);
                    acc[tt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[tt], 0, 0, 0);
                }
            }
        }
    }
    // D: lane holds rows 4kq+i, output channel co0+16tt+m
#pragma unroll
    for (int tt = 0; tt < 4; ++tt) {
        if (tt >= ntile) continue;
        const int co = co0 + 16 * tt + m;
        const float b = A.bias ? A.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + 4 * kq + i;
            if (r >= rows) continue;
            const int64_t dv = dst_voxel<I>(A, r, p);
            float v = acc[tt][i] + b;
            if (A.out_bf) {
                if (A.act) v = v > 0.f ? v : A.slope * v;
                A.out_bf[dv * A.Cout + co] = f2bf(v);
            } else {
                float* dst = co < A.Csplit ? A.out_f + dv * A.Csplit + co
                                           : A.out_f2 + dv * (A.Cout - A.Csplit) + (co - A.Csplit);
                *dst = A.accumulate ? *dst + v : v;
            }
        }
    }
}

// 3x3x3 convolution (stride 1, zero padding) as an implicit GEMM with its
// input staged in LDS.  A workgroup of 4 waves owns an output brick of 8x8x4
// voxels of one sample and 16 NT output channels (blockIdx.y); wave w owns the
// brick's z-plane w: 64 rows in 4 MFMA row tiles (row = 8 y + x).  The
// reduction runs over taps x input channels in chunks of CC = min(Cin, 32)
// channels: the chunk's 10x10x6 halo brick is loaded once (zero outside the
// grid) and every tap reads it from LDS; one K = 32 step covers one tap of a
// 32-channel chunk or two taps of a 16-channel chunk (tap 27 is zero).  A
// lane's 8 K values are 8 consecutive channels of one voxel: one 16-byte LDS
// read.  The weights' B fragments (8 consecutive input channels of one tap and
// output channel) come from global memory, shared by the 4 row tiles.
constexpr int kHalo3 = 10 * 10 * 6;

template <int NT>
__global__ void __launch_bounds__(256) k_conv3(ConvArgs A, int nbx, int nbz) {
    extern __shared__ uint4 hal[];  // [kHalo3][CC / 8]
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int D = A.Dout;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nbx;
    b /= nbx;
    const int bz = b % nbz;
    const int n = b / nbz;
    const int x0 = 8 * bx, y0 = 8 * by, z0 = 4 * bz;
    const int co0 = blockIdx.y * 16 * NT;
    const int Cin = A.C1 + A.C2;
    const int CC = Cin < 32 ? Cin : 32;
    const int oct = CC >> 3;
    const int m = lane & 15, kq = lane >> 4;
    f32x4 acc[4][NT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[r][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    const int ksteps = (27 * CC + 31) / 32;
    for (int c0 = 0; c0 < Cin; c0 += CC) {
        __syncthreads();
        for (int i = threadIdx.x; i < kHalo3 * oct; i += 256) {
            const int o = i % oct, hv = i / oct;
            const int hx = hv % 10, hy = (hv / 10) % 10, hz = hv / 100;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = {0u, 0u, 0u, 0u};
            if ((unsigned)gx < (unsigned)D && (unsigned)gy < (unsigned)D && (unsigned)gz < (unsigned)D) {
                const int64_t sv = (((int64_t)n * D + gz) * D + gy) * D + gx;
                const int c = c0 + 8 * o;
                const uint16_t* src = c < A.C1 ? A.in1 + sv * A.C1 + c : A.in2 + sv * A.C2 + (c - A.C1);
                v = *reinterpret_cast<const uint4*>(src);
            }
            hal[i] = v;
        }
        __syncthreads();
        for (int s = 0; s < ksteps; ++s) {
            const int k = 32 * s + 8 * kq;
            const int t = k / CC, c = k - t * CC;
            const bool tap_ok = t < 27;
            uint4 bw[NT];
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                bw[tt] = (uint4){0u, 0u, 0u, 0u};
                if (tap_ok)
                    bw[tt] = *reinterpret_cast<const uint4*>(A.w + ((size_t)t * A.Cout + co0 + 16 * tt + m) * Cin +
                                                             c0 + c);
            }
            const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;  // offsets + 1
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                uint4 a = {0u, 0u, 0u, 0u};
                if (tap_ok) {
                    const int hx = (m & 7) + dx, hy = 2 * r + (m >> 3) + dy, hz = wave + dz;
                    a = hal[((hz * 10 + hy) * 10 + hx) * oct + (c >> 3)];
                }
#pragma unroll
                for (int tt = 0; tt < NT; ++tt) acc[r][tt] = mfma32(a, bw[tt], acc[r][tt]);
            }
        }
    }
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
        const int co = co0 + 16 * tt + m;
        const float bias = A.bias ? A.bias[co] : 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = 4 * kq + i;  // row within the tile: x = rr % 8, y = 2 r + rr / 8
                const int64_t dv = (((int64_t)n * D + z0 + wave) * D + y0 + 2 * r + (rr >> 3)) * D + x0 + (rr & 7);
                float v = acc[r][tt][i] + bias;
                if (A.out_bf) {
                    if (A.act) v = v > 0.f ? v : A.slope * v;
                    A.out_bf[dv * A.Cout + co] = f2bf(v);
                } else {
                    float* dst = co < A.Csplit ? A.out_f + dv * A.Csplit + co
                                               : A.out_f2 + dv * (A.Cout - A.Csplit) + (co - A.Csplit);
                    *dst = A.accumulate ? *dst + v : v;
                }
            }
        }
    }
}

struct WgradArgs {
    const uint16_t* x1;   // layer input(s) [N][Din^3][C1], [N][Din^3][C2]
    const uint16_t* x2;
    int C1, C2;
    const uint16_t* dz;   // gradient at the layer's pre-activation [N][Dout^3][Cout]
    int Cout;
    int N, Din, Dout, mode;
    float* dw;            // [taps][Cout][C1+C2], accumulated
};

// dW[t][co][ci] += sum over rows of dz[dst(row)][co] * x[src(row, t)][ci].
// MFMA with M = output channels, N = input channels, K = rows.  Each wave
// reduces `chunk` rows for one (tap, 16x16 channel tile) and adds its tile to
// dW with FP32 atomics.
template <typename I>
__global__ void __launch_bounds__(256) k_wgrad(WgradArgs W, int64_t rows, int chunk) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int Cin = W.C1 + W.C2;
    const int ct_in = Cin / 16, ct_out = W.Cout / 16;
    const int taps = W.mode == CONV3 ? 27 : 8;
    const int64_t task = (int64_t)blockIdx.y * 4 + wave;  // (tap, co tile, ci tile)
    if (task >= (int64_t)taps * ct_out * ct_in) return;
    const int t = (int)(task / (ct_out * ct_in));
    const int rem = (int)(task - (int64_t)t * ct_out * ct_in);
    const int cot = rem / ct_in, cit = rem - cot * ct_in;
    ConvArgs G{};
    G.C1 = W.C1;
    G.C2 = W.C2;
    G.N = W.N;
    G.Din = W.Din;
    G.Dout = W.Dout;
    G.mode = W.mode;
    const int m = lane & 15, kq = lane >> 4;
    const int co = cot * 16 + m;  // A row (output channel), B column index uses m as ci
    const int ci = cit * 16 + m;
    const int64_t rbeg = (int64_t)blockIdx.x * chunk;
    const int64_t rend = min(rows, rbeg + chunk);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t r0 = rbeg; r0 < rend; r0 += 16) {
        bf16x4 a, b;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t r = r0 + 4 * kq + i;
            uint16_t av = 0, bv = 0;
            if (r < rend) {
                int64_t dv, sv;
                if (W.mode == UP) {  // row = input voxel u, tap t = parity of the output voxel
                    sv = r;
                    dv = dst_voxel<I>(G, r, t);
                } else {
                    dv = r;
                    sv = src_voxel<I>(G, r, t);
                }
                av = W.dz[dv * W.Cout + co];
                if (sv >= 0)
                    bv = ci < W.C1 ? W.x1[sv * W.C1 + ci] : W.x2[sv * W.C2 + (ci - W.C1)];
            }
            a[i] = (short)av;
            b[i] = (short)bv;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    // D[m' = co tile row 4kq+i][n = ci m]
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int coo = cot * 16 + 4 * kq + i;
        atomicAdd(W.dw + ((size_t)t * W.Cout + coo) * Cin + ci, acc[i]);
    }
}

// Weight gradients of a 3x3x3 convolution with LDS-staged operands:
// dW[t][co][ci] += sum over output voxels v of dz[v][co] x[v + delta_t][ci].
// A workgroup owns a column of 8x8x8 bricks of one sample (all z), a
// 16-channel slice of the input (blockIdx.y) and 16 NCO output channels
// (blockIdx.z).  Per brick, dz is staged transposed ([co][voxel], so that a
// lane's 8 K values, 8 consecutive voxels of one x-line, are one 16-byte
// read) and x with its halo channels-last.  MFMA 16x16x32: M = output channel,
// N = input channel, K = 32 voxels (four x-lines); wave w owns taps w, w + 4,
// ... and keeps their tiles in registers across the column; one FP32 atomic
// add per weight and workgroup at the end.
constexpr int kDzStride = 520;  // 512 voxels + 8: consecutive channels 16 B apart in bank order

template <int NCO>
__global__ void __launch_bounds__(256) k_wgrad3(WgradArgs W, int nbx) {
    __shared__ __align__(16) uint16_t dzT[16 * NCO][kDzStride];
    __shared__ __align__(16) uint16_t xh[1000 * 16];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int D = W.Dout;
    int b = blockIdx.x;
    const int bx = b % nbx;
    b /= nbx;
    const int by = b % nbx;
    const int n = b / nbx;
    const int x0 = 8 * bx, y0 = 8 * by;
    const int ci0 = blockIdx.y * 16, co0 = blockIdx.z * 16 * NCO;
    const int Cin = W.C1 + W.C2;
    const int m = lane & 15, kq = lane >> 4;
    f32x4 acc[7][NCO];
#pragma unroll
    for (int j = 0; j < 7; ++j)
#pragma unroll
        for (int t = 0; t < NCO; ++t) acc[j][t] = (f32x4){0.f, 0.f, 0.f, 0.f};
    for (int z0 = 0; z0 < D; z0 += 8) {
        __syncthreads();
        // dz of the brick: 512 voxels x 2 NCO octets, written transposed
        for (int i = threadIdx.x; i < 512 * 2 * NCO; i += 256) {
            const int o = i % (2 * NCO), v = i / (2 * NCO);
            const int64_t gv = (((int64_t)n * D + z0 + (v >> 6)) * D + y0 + ((v >> 3) & 7)) * D + x0 + (v & 7);
            const s16x8 q = *reinterpret_cast<const s16x8*>(W.dz + gv * W.Cout + co0 + 8 * o);
#pragma unroll
            for (int j = 0; j < 8; ++j) dzT[8 * o + j][v] = (uint16_t)q[j];
        }
        // x slice with its halo: 10x10x10 voxels x 2 octets
        for (int i = threadIdx.x; i < 2000; i += 256) {
            const int o = i & 1, hv = i >> 1;
            const int hx = hv % 10, hy = (hv / 10) % 10, hz = hv / 100;
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 v = {0u, 0u, 0u, 0u};
            if ((unsigned)gx < (unsigned)D && (unsigned)gy < (unsigned)D && (unsigned)gz < (unsigned)D) {
                const int64_t sv = (((int64_t)n * D + gz) * D + gy) * D + gx;
                const int c = ci0 + 8 * o;
                const uint16_t* src = c < W.C1 ? W.x1 + sv * W.C1 + c : W.x2 + sv * W.C2 + (c - W.C1);
                v = *reinterpret_cast<const uint4*>(src);
            }
            *reinterpret_cast<uint4*>(xh + hv * 16 + 8 * o) = v;
        }
        __syncthreads();
        for (int kg = 0; kg < 16; ++kg) {
            const int z = kg >> 1, y = 4 * (kg & 1) + kq;  // this lane's x-line
            uint4 a[NCO];
#pragma unroll
            for (int tt = 0; tt < NCO; ++tt)
                a[tt] = *reinterpret_cast<const uint4*>(&dzT[16 * tt + m][z * 64 + y * 8]);
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int t = wave + 4 * j;
                if (t < 27) {
                    const int dz = t / 9, dy = (t / 3) % 3, dx = t % 3;  // offsets + 1
                    const uint16_t* xs = xh + (((z + dz) * 10 + y + dy) * 10 + dx) * 16 + m;
                    s16x8 q;
#pragma unroll
                    for (int i = 0; i < 8; ++i) q[i] = (short)xs[16 * i];
                    const uint4 bq = __builtin_bit_cast(uint4, q);
#pragma unroll
                    for (int tt = 0; tt < NCO; ++tt) acc[j][tt] = mfma32(a[tt], bq, acc[j][tt]);
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int t = wave + 4 * j;
        if (t >= 27) continue;
#pragma unroll
        for (int tt = 0; tt < NCO; ++tt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int co = co0 + 16 * tt + 4 * kq + i;
                atomicAdd(W.dw + ((size_t)t * W.Cout + co) * Cin + ci0 + m, acc[j][tt][i]);
            }
    }
}

// dz = dy * LeakyReLU'(y) as BF16 (y is the layer's post-activation output,
// whose sign equals the pre-activation's), plus the bias gradient.  C divides
// the block size and the grid stride (C a power of two <= 256, blocks of 256
// threads), so a thread only ever sees channel threadIdx.x % C: it sums its
// channel in a register and adds it once.
__global__ void k_act_back(int64_t n, int C, const float* __restrict__ dy,
                           const uint16_t* __restrict__ y, float slope, int act,
                           uint16_t* __restrict__ dz, float* __restrict__ dbias) {
    __shared__ float sb[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sb[i] = 0.f;
    __syncthreads();
    float acc = 0.f;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        float g = dy[j];
        if (act && !(bf2f(y[j]) > 0.f)) g *= slope;
        dz[j] = f2bf(g);
        acc += g;
    }
    atomicAdd(&sb[threadIdx.x % C], acc);
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) atomicAdd(dbias + c, sb[c]);
}

// The same, eight consecutive elements per thread with 16-byte loads and
// stores (n a multiple of 8, 16-byte aligned arrays, 8 <= C): element 8 j + k
// has channel (8 threadIdx.x + k) mod C, so a thread sums the same eight
// channels throughout.
__global__ void k_act_back8(int64_t n8, int C, const float4* __restrict__ dy,
                            const uint4* __restrict__ y, float slope, int act, uint4* __restrict__ dz,
                            float* __restrict__ dbias) {
    __shared__ float sb[256];
    for (int i = threadIdx.x; i < 256; i += blockDim.x) sb[i] = 0.f;
    __syncthreads();
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n8;
         j += (int64_t)gridDim.x * blockDim.x) {
        const float4 a = dy[2 * j], b = dy[2 * j + 1];
        const uint4 yy = y[j];
        float g[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        const uint32_t yw[4] = {yy.x, yy.y, yy.z, yy.w};
        uint32_t o[4];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint16_t yk = (uint16_t)(yw[k >> 1] >> (16 * (k & 1)));
            if (act && !(bf2f(yk) > 0.f)) g[k] *= slope;
            acc[k] += g[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) o[k] = (uint32_t)f2bf(g[2 * k]) | ((uint32_t)f2bf(g[2 * k + 1]) << 16);
        dz[j] = make_uint4(o[0], o[1], o[2], o[3]);
    }
    const int base = (8 * threadIdx.x) % C;
#pragma unroll
    for (int k = 0; k < 8; ++k) atomicAdd(&sb[base + k], acc[k]);
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) atomicAdd(dbias + c, sb[c]);
}

// Input layer: the NF = 3 FP32 features of each voxel [N][V][3], shifted and
// scaled to O(1), as BF16 channels-last with 16 channels (zero padded).
__global__ void k_pack_input(int64_t nvox, const float* __restrict__ x, uint16_t* __restrict__ out,
                             float sh0, float sc0, float sh1, float sc1, float sh2, float sc2) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        uint16_t* o = out + v * 16;
        o[0] = f2bf((x[3 * v] + sh0) * sc0);
        o[1] = f2bf((x[3 * v + 1] + sh1) * sc1);
        o[2] = f2bf((x[3 * v + 2] + sh2) * sc2);
#pragma unroll
        for (int c = 3; c < 16; ++c) o[c] = 0;
    }
}

// 1x1x1 head, C -> 1 channel, FP32 output: y[v] = sum_c w[c] x[v][c] + b
template <int C>
__global__ void k_head(int64_t nvox, const uint16_t* __restrict__ x, const float* __restrict__ w,
                       const float* __restrict__ b, float* __restrict__ y) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        float s = b[0];
#pragma unroll
        for (int c = 0; c < C; ++c) s += w[c] * bf2f(x[v * C + c]);
        y[v] = s;
    }
}

// masked mean-square loss of the prediction: loss += sum mask (y - t)^2;
// dy = 2 mask (y - t) / count
__global__ void k_loss(int64_t nvox, const float* __restrict__ y, const float* __restrict__ t,
                       const float* __restrict__ mask, float inv_count, float* __restrict__ dy,
                       double* loss) {
    __shared__ double s[256];
    double acc = 0.0;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float d = (y[v] - t[v]) * mask[v];
        acc += (double)d * d;
        dy[v] = 2.f * d * inv_count;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(loss, s[0]);
}

// head backward: dw[c] += sum dy[v] x[v][c]; db += sum dy; dx[v][c] = dy[v] w[c]
template <int C>
__global__ void k_head_back(int64_t nvox, const uint16_t* __restrict__ x, const float* __restrict__ w,
                            const float* __restrict__ dy, float* __restrict__ dw,
                            float* __restrict__ db, float* __restrict__ dx) {
    __shared__ float s[C + 1];
    if (threadIdx.x <= C) s[threadIdx.x] = 0.f;
    __syncthreads();
    float lw[C], lb = 0.f;
#pragma unroll
    for (int c = 0; c < C; ++c) lw[c] = 0.f;
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        const float g = dy[v];
        lb += g;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            lw[c] += g * bf2f(x[v * C + c]);
            dx[v * C + c] = g * w[c];
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) atomicAdd(&s[c], lw[c]);
    atomicAdd(&s[C], lb);
    __syncthreads();
    if (threadIdx.x < C) atomicAdd(dw + threadIdx.x, s[threadIdx.x]);
    if (threadIdx.x == C) atomicAdd(db, s[C]);
}

// Adam on the FP32 master parameters (bias-corrected moments; c1, c2 are
// 1/(1 - b1^step), 1/(1 - b2^step)).

// Sum of squares of the gradient (for clipping by global norm).
__global__ void k_sumsq(int64_t n, const float* __restrict__ g, double* out) {
    __shared__ double s[256];
    double a = 0.0;
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x)
        a += (double)g[j] * g[j];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(out, s[0]);
}

// gradients are scaled by min(1, clip / ||g||) when clip > 0 (sumsq on device)
__global__ void k_adam(int64_t n, float* __restrict__ p, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2, float clip, const double* __restrict__ sumsq) {
    float scale = 1.f;
    if (clip > 0.f) {
        const double nrm = sqrt(*sumsq);
        if (nrm > (double)clip) scale = (float)((double)clip / nrm);
    }
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const float gj = g[j] * scale;
        const float mj = b1 * m[j] + (1.f - b1) * gj;
        const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
        m[j] = mj;
        v[j] = vj;
        p[j] -= lr * (mj * c1) / (sqrtf(vj * c2) + eps);
    }
}

// BF16 copies of one layer's weights: w16 = p, wt16[t'][ci][co] = p[t][co][ci]
// with t' = 26 - t for CONV3 (flipped taps) and t' = t otherwise.
__global__ void k_weights_bf16(int64_t n, const float* __restrict__ p, int taps, int Cout, int Cin,
                               int conv3, uint16_t* __restrict__ w16, uint16_t* __restrict__ wt16) {
    for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(j / ((int64_t)Cout * Cin));
        const int r = (int)(j - (int64_t)t * Cout * Cin);
        const int co = r / Cin, ci = r - co * Cin;
        const uint16_t h = f2bf(p[j]);
        w16[j] = h;
        const int tt = conv3 ? taps - 1 - t : t;
        wt16[((int64_t)tt * Cin + ci) * Cout + co] = h;
    }
}

// Features of the warm start per cell v (cell coordinates i, j, k):
//   x[v][0] = log10 max(rho chi(1 um) dx, 1e-6)  (optical depth of one cell width)
//   x[v][1] = log10(D_v + 1e-30), D the deposit field: luminosity of the
//             sources in the cell / (4 pi dx^2), erg s^-1 cm^-2
//   x[v][2] = log10(sum_c D_c dx^2 / max(r_vc^2, dx^2/4) + 1e-30): the deposit
//             field spread by the free-space kernel 1/r^2 (r between cell
//             centres), i.e. the unattenuated flux of the deposited luminosity.
// The nd deposit cells are listed as (i, j, k, D).
__global__ void k_features(int64_t nvox, int nx, int ny, const double* __restrict__ rho,
                           double chi1_dx, const double* __restrict__ dep, const int* __restrict__ dcell,
                           const double* __restrict__ dval, int nd, float* __restrict__ x) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < nvox;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double tau = rho[v] * chi1_dx;
        x[3 * v] = (float)log10(tau > 1e-6 ? tau : 1e-6);
        x[3 * v + 1] = (float)log10(dep[v] + 1e-30);
        const int i = (int)(v % nx), j = (int)((v / nx) % ny), k = (int)(v / ((int64_t)nx * ny));
        double f = 0.0;
        for (int q = 0; q < nd; ++q) {
            const double a = i - dcell[3 * q], b = j - dcell[3 * q + 1], c = k - dcell[3 * q + 2];
            const double r2 = a * a + b * b + c * c;
            f += dval[q] / (r2 > 0.25 ? r2 : 0.25);
        }
        x[3 * v + 2] = (float)log10(f + 1e-30);
    }
}

// T = 10^y (bounded to the temperature range of the solver)
__global__ void k_exp10(int64_t n, const float* __restrict__ y, double* __restrict__ T) {
    for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < n;
         v += (int64_t)gridDim.x * blockDim.x) {
        const double t = pow(10.0, (double)y[v]);
        T[v] = t < 1.0 ? 1.0 : (t > 1e4 ? 1e4 : t);
    }
}

// ---------------------------------------------------------------------------
// whether every voxel index of a layer (N samples, grids Din and Dout) fits 32 bits
static bool index32(int N, int Din, int Dout) {
    const int64_t d = Din > Dout ? Din : Dout;
    return (int64_t)N * d * d * d < ((int64_t)1 << 32);
}

static int blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (int)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
}

hipError_t launch_conv(const ConvArgs& A, hipStream_t st) {
    if (A.mode == CONV3 && A.Din == A.Dout && A.Dout % 8 == 0 && A.Cout % 16 == 0 &&
        (A.C1 + A.C2) % 16 == 0 && A.C1 % 16 == 0) {
        const int nbx = A.Dout / 8, nbz = A.Dout / 4;
        const int cin = A.C1 + A.C2;
        const size_t lds = (size_t)kHalo3 * (cin < 32 ? cin : 32) * 2;
        const int nt = A.Cout % 64 == 0 ? 4 : (A.Cout % 32 == 0 ? 2 : 1);
        dim3 grid((unsigned)(nbx * nbx * nbz * A.N), (unsigned)(A.Cout / (16 * nt)));
        if (nt == 4)
            hipLaunchKernelGGL(k_conv3<4>, grid, dim3(256), lds, st, A, nbx, nbz);
        else if (nt == 2)
            hipLaunchKernelGGL(k_conv3<2>, grid, dim3(256), lds, st, A, nbx, nbz);
        else
            hipLaunchKernelGGL(k_conv3<1>, grid, dim3(256), lds, st, A, nbx, nbz);
        return hipGetLastError();
    }
    // rows of the GEMM: output voxels (CONV3, DOWN) or input voxels (UP)
    const int Dg = A.mode == UP ? A.Din : A.Dout;
    const int64_t rows = (int64_t)A.N * Dg * Dg * Dg;
    dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((A.Cout + 63) / 64), A.mode == UP ? 8 : 1);
    if (index32(A.N, A.Din, A.Dout))
        hipLaunchKernelGGL(k_conv<uint32_t>, grid, dim3(256), 0, st, A, rows);
    else
        hipLaunchKernelGGL(k_conv<int64_t>, grid, dim3(256), 0, st, A, rows);
    return hipGetLastError();
}

hipError_t launch_wgrad(const WgradArgs& W, hipStream_t st) {
    if (W.mode == CONV3 && W.Din == W.Dout && W.Dout % 8 == 0 && W.Cout % 16 == 0 &&
        W.C1 % 16 == 0 && W.C2 % 16 == 0) {
        const int nbx = W.Dout / 8;
        const int nco = W.Cout % 32 == 0 ? 2 : 1;
        dim3 grid((unsigned)(nbx * nbx * W.N), (unsigned)((W.C1 + W.C2) / 16), (unsigned)(W.Cout / (16 * nco)));
        if (nco == 2)
            hipLaunchKernelGGL(k_wgrad3<2>, grid, dim3(256), 0, st, W, nbx);
        else
            hipLaunchKernelGGL(k_wgrad3<1>, grid, dim3(256), 0, st, W, nbx);
        return hipGetLastError();
    }
    const int Dg = W.mode == UP ? W.Din : W.Dout;
    const int64_t rows = (int64_t)W.N * Dg * Dg * Dg;
    const int taps = W.mode == CONV3 ? 27 : 8;
    const int64_t tasks = (int64_t)taps * (W.Cout / 16) * ((W.C1 + W.C2) / 16);
    // rows per wave: enough that the grid holds about 4096 workgroups (fewer
    // FP32 atomics per weight), a multiple of 16, at least 256
    const int64_t gy = (tasks + 3) / 4;
    int64_t c = (rows * gy + 4095) / 4096;
    c = (c + 15) / 16 * 16;
    if (c < 256) c = 256;
    if (c > (1 << 20)) c = 1 << 20;
    const int chunk = (int)c;
    dim3 grid((unsigned)((rows + chunk - 1) / chunk), (unsigned)((tasks + 3) / 4));
    if (index32(W.N, W.Din, W.Dout))
        hipLaunchKernelGGL(k_wgrad<uint32_t>, grid, dim3(256), 0, st, W, rows, chunk);
    else
        hipLaunchKernelGGL(k_wgrad<int64_t>, grid, dim3(256), 0, st, W, rows, chunk);
    return hipGetLastError();
}

hipError_t launch_act_back(int64_t n, int C, const float* dy, const uint16_t* y, float slope, int act,
                           uint16_t* dz, float* dbias, hipStream_t st) {
    if (C < 1 || C > 256 || (C & (C - 1)) != 0) return hipErrorInvalidValue;
    const bool vec = C >= 8 && n % 8 == 0 && ((uintptr_t)dy | (uintptr_t)y | (uintptr_t)dz) % 16 == 0;
    // at most 512 groups: every group ends with one FP32 atomic per channel on
    // the same C addresses, which serialise (4096 groups: 4096 per address,
    // the larger part of a small layer's time)
    if (vec)
        hipLaunchKernelGGL(k_act_back8, dim3(std::min(blocks_for(n / 8), 512)), dim3(256), 0, st, n / 8, C,
                           reinterpret_cast<const float4*>(dy), reinterpret_cast<const uint4*>(y), slope,
                           act, reinterpret_cast<uint4*>(dz), dbias);
    else
        hipLaunchKernelGGL(k_act_back, dim3(blocks_for(n)), dim3(256), 0, st, n, C, dy, y, slope, act, dz,
                           dbias);
    return hipGetLastError();
}
hipError_t launch_pack_input(int64_t nvox, const float* x, uint16_t* out, const float* norm,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_pack_input, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, x, out, norm[0],
                       norm[1], norm[2], norm[3], norm[4], norm[5]);
    return hipGetLastError();
}
hipError_t launch_head(int C, int64_t nvox, const uint16_t* x, const float* w, const float* b, float* y,
                       hipStream_t st) {
    if (C == 16)
        hipLaunchKernelGGL(k_head<16>, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, x, w, b, y);
    else if (C == 32)
        hipLaunchKernelGGL(k_head<32>, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, x, w, b, y);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
hipError_t launch_loss(int64_t nvox, const float* y, const float* t, const float* mask,
                       float inv_count, float* dy, double* loss, hipStream_t st) {
    hipLaunchKernelGGL(k_loss, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, y, t, mask, inv_count,
                       dy, loss);
    return hipGetLastError();
}
hipError_t launch_head_back(int C, int64_t nvox, const uint16_t* x, const float* w, const float* dy,
                            float* dw, float* db, float* dx, hipStream_t st) {
    if (C == 16)
        hipLaunchKernelGGL(k_head_back<16>, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, x, w, dy,
                           dw, db, dx);
    else if (C == 32)
        hipLaunchKernelGGL(k_head_back<32>, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, x, w, dy,
                           dw, db, dx);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2, float clip, double* sumsq,
                       hipStream_t st) {
    if (clip > 0.f)
        hipLaunchKernelGGL(k_sumsq, dim3(blocks_for(n)), dim3(256), 0, st, n, g, sumsq);
    hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps,
                       c1, c2, clip, (const double*)sumsq);
    return hipGetLastError();
}
hipError_t launch_weights_bf16(int64_t n, const float* p, int taps, int Cout, int Cin, int conv3,
                               uint16_t* w16, uint16_t* wt16, hipStream_t st) {
    hipLaunchKernelGGL(k_weights_bf16, dim3(blocks_for(n)), dim3(256), 0, st, n, p, taps, Cout, Cin,
                       conv3, w16, wt16);
    return hipGetLastError();
}
hipError_t launch_features(int64_t nvox, int nx, int ny, const double* rho, double chi1_dx,
                           const double* dep, const int* dcell, const double* dval, int nd, float* x,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_features, dim3(blocks_for(nvox)), dim3(256), 0, st, nvox, nx, ny, rho, chi1_dx,
                       dep, dcell, dval, nd, x);
    return hipGetLastError();
}
hipError_t launch_exp10(int64_t n, const float* y, double* T, hipStream_t st) {
    hipLaunchKernelGGL(k_exp10, dim3(blocks_for(n)), dim3(256), 0, st, n, y, T);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace mcrt
