// mcrt_surrogate.cpp -- host side of the learned warm start: a 4-level 3-D
// convolutional encoder-decoder (channels C0, 2C0, 4C0, 8C0; two 3x3x3
// convolutions per level; stride-2 2x2x2 down and transposed up
// convolutions; skip concatenation; 1x1x1 head) that maps per-cell features
// (cell optical depth, source luminosity deposit, the deposit spread by
// 1/r^2) to log10 T.  Weights are
// FP32 masters updated by Adam with BF16 copies for the matrix cores.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <random>
#include <string>
#include <vector>

#include "../../include/mcrt.h"

namespace mcrt {
namespace nn {
enum Mode : int { CONV3 = 0, DOWN = 1, UP = 2 };
struct ConvArgs {
    const uint16_t* in1;
    const uint16_t* in2;
    int C1, C2;
    const uint16_t* w;
    const float* bias;
    int Cout;
    int N, Din, Dout;
    int mode;
    uint16_t* out_bf;
    float* out_f;
    float* out_f2;
    int Csplit;
    int act;
    float slope;
    int accumulate;
};
struct WgradArgs {
    const uint16_t* x1;
    const uint16_t* x2;
    int C1, C2;
    const uint16_t* dz;
    int Cout;
    int N, Din, Dout, mode;
    float* dw;
};
hipError_t launch_conv(const ConvArgs& A, hipStream_t st);
hipError_t launch_wgrad(const WgradArgs& W, hipStream_t st);
hipError_t launch_act_back(int64_t n, int C, const float* dy, const uint16_t* y, float slope, int act,
                           uint16_t* dz, float* dbias, hipStream_t st);
hipError_t launch_pack_input(int64_t nvox, const float* x, uint16_t* out, const float* norm,
                             hipStream_t st);
hipError_t launch_head(int C, int64_t nvox, const uint16_t* x, const float* w, const float* b, float* y,
                       hipStream_t st);
hipError_t launch_loss(int64_t nvox, const float* y, const float* t, const float* mask,
                       float inv_count, float* dy, double* loss, hipStream_t st);
hipError_t launch_head_back(int C, int64_t nvox, const uint16_t* x, const float* w, const float* dy,
                            float* dw, float* db, float* dx, hipStream_t st);
hipError_t launch_adam(int64_t n, float* p, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2, float clip, double* sumsq,
                       hipStream_t st);
hipError_t launch_weights_bf16(int64_t n, const float* p, int taps, int Cout, int Cin, int conv3,
                               uint16_t* w16, uint16_t* wt16, hipStream_t st);
hipError_t launch_exp10(int64_t n, const float* y, double* T, hipStream_t st);
}  // namespace nn
}  // namespace mcrt

using namespace mcrt::nn;

namespace {

constexpr float kSlope = 0.1f;  // LeakyReLU
// input scaling: channel 0 (log10 cell optical depth, -6..2) -> (x + 2) / 2,
// channel 1 (log10 deposit field, -30 outside source cells) -> (x + 30) / 10,
// channel 2 (log10 spread deposit field, about 0..10) -> (x - 4) / 3
constexpr float kNorm[6] = {2.f, 0.5f, 30.f, 0.1f, -4.f, 1.f / 3.f};

struct Layer {
    int mode;
    int in1, in2;        // tensor ids (in2 = -1: no concatenation)
    int out;             // tensor id
    int C1, C2, Cout;
    int Din, Dout;       // relative grid divisors: side = D >> level
    int lin, lout;       // levels of input and output grids
    int64_t woff, boff;  // offsets in the parameter array
    int taps;
    int64_t nw() const { return (int64_t)taps * Cout * (C1 + C2); }
};

struct Tensor {
    int C;
    int level;
    uint16_t* y = nullptr;  // BF16 activations
    float* g = nullptr;     // FP32 gradient
    size_t cap = 0;         // elements allocated
};

}  // namespace

struct mcrt_surrogate {
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int C0 = 16;
    std::vector<Layer> layers;
    std::vector<Tensor> tensors;
    int64_t nparam = 0, head_w = 0, head_b = 0;
    float* p = nullptr;      // FP32 master parameters
    float* gp = nullptr;     // gradients
    float* m1 = nullptr;     // Adam moments
    float* m2 = nullptr;
    uint16_t* w16 = nullptr; // BF16 forward weights (same offsets as p)
    uint16_t* wt16 = nullptr;// BF16 backward-data weights
    int64_t step = 0;
    double grad_clip = 0.0;  // global-norm clipping of the gradient (0: off)
    // per-call buffers
    float* pred = nullptr;
    float* dpred = nullptr;
    uint16_t* dz = nullptr;
    double* loss = nullptr;   // [0] loss, [1] gradient sum of squares
    size_t cap_vox = 0, cap_dz = 0;
};

namespace {

mcrt_status sfail(mcrt_surrogate* s, mcrt_status st, const std::string& msg) {
    s->err = msg;
    return st;
}

#define SCHK(expr)                                                                           \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return sfail(s, e_ == hipErrorOutOfMemory ? MCRT_E_NOMEM : MCRT_E_DEVICE,        \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

void build_net(mcrt_surrogate* s) {
    const int C0 = s->C0;
    auto tensor = [&](int C, int level) {
        Tensor t;
        t.C = C;
        t.level = level;
        s->tensors.push_back(t);
        return (int)s->tensors.size() - 1;
    };
    int64_t off = 0;
    auto layer = [&](int mode, int in1, int in2, int Cout, int lout) {
        Layer L;
        L.mode = mode;
        L.in1 = in1;
        L.in2 = in2;
        L.C1 = s->tensors[in1].C;
        L.C2 = in2 >= 0 ? s->tensors[in2].C : 0;
        L.Cout = Cout;
        L.lin = s->tensors[in1].level;
        L.lout = lout;
        L.taps = mode == CONV3 ? 27 : 8;
        L.out = tensor(Cout, lout);
        L.woff = off;
        off += L.nw();
        L.boff = off;
        off += Cout;
        s->layers.push_back(L);
        return L.out;
    };
    const int x = tensor(16, 0);  // 2 feature channels zero-padded to 16
    int t = layer(CONV3, x, -1, C0, 0);
    const int s0 = layer(CONV3, t, -1, C0, 0);
    t = layer(DOWN, s0, -1, 2 * C0, 1);
    t = layer(CONV3, t, -1, 2 * C0, 1);
    const int s1 = layer(CONV3, t, -1, 2 * C0, 1);
    t = layer(DOWN, s1, -1, 4 * C0, 2);
    t = layer(CONV3, t, -1, 4 * C0, 2);
    const int s2 = layer(CONV3, t, -1, 4 * C0, 2);
    t = layer(DOWN, s2, -1, 8 * C0, 3);
    t = layer(CONV3, t, -1, 8 * C0, 3);
    t = layer(CONV3, t, -1, 8 * C0, 3);
    t = layer(UP, t, -1, 4 * C0, 2);
    t = layer(CONV3, t, s2, 4 * C0, 2);
    t = layer(CONV3, t, -1, 4 * C0, 2);
    t = layer(UP, t, -1, 2 * C0, 1);
    t = layer(CONV3, t, s1, 2 * C0, 1);
    t = layer(CONV3, t, -1, 2 * C0, 1);
    t = layer(UP, t, -1, C0, 0);
    t = layer(CONV3, t, s0, C0, 0);
    t = layer(CONV3, t, -1, C0, 0);
    s->head_w = off;
    off += C0;
    s->head_b = off;
    off += 1;
    s->nparam = off;
}

mcrt_status refresh_bf16(mcrt_surrogate* s) {
    for (const Layer& L : s->layers)
        SCHK(launch_weights_bf16(L.nw(), s->p + L.woff, L.taps, L.Cout, L.C1 + L.C2, L.mode == CONV3,
                                 s->w16 + L.woff, s->wt16 + L.woff, s->stream));
    return MCRT_OK;
}

mcrt_status ensure_buffers(mcrt_surrogate* s, int N, int D, bool train) {
    const int64_t vox = (int64_t)N * D * D * D;
    for (Tensor& t : s->tensors) {
        const int side = D >> t.level;
        const size_t n = (size_t)N * side * side * side * t.C;
        if (n > t.cap) {
            if (t.y) hipFree(t.y);
            if (t.g) hipFree(t.g);
            t.y = nullptr;
            t.g = nullptr;
            SCHK(hipMalloc((void**)&t.y, n * sizeof(uint16_t)));
            t.cap = n;
        }
        if (train && !t.g) SCHK(hipMalloc((void**)&t.g, t.cap * sizeof(float)));
    }
    if ((size_t)vox > s->cap_vox) {
        if (s->pred) hipFree(s->pred);
        if (s->dpred) hipFree(s->dpred);
        SCHK(hipMalloc((void**)&s->pred, vox * sizeof(float)));
        SCHK(hipMalloc((void**)&s->dpred, vox * sizeof(float)));
        s->cap_vox = (size_t)vox;
    }
    if (train) {
        size_t mx = 0;
        for (const Tensor& t : s->tensors) mx = std::max(mx, t.cap);
        if (mx > s->cap_dz) {
            if (s->dz) hipFree(s->dz);
            SCHK(hipMalloc((void**)&s->dz, mx * sizeof(uint16_t)));
            s->cap_dz = mx;
        }
    }
    return MCRT_OK;
}

mcrt_status check_shape(mcrt_surrogate* s, int N, int D) {
    if (N < 1 || D < 8 || D % 8 != 0) return sfail(s, MCRT_E_ARG, "grid side must be a multiple of 8");
    return MCRT_OK;
}

mcrt_status forward(mcrt_surrogate* s, const float* d_x, int N, int D) {
    hipStream_t st = s->stream;
    const int64_t vox = (int64_t)N * D * D * D;
    SCHK(launch_pack_input(vox, d_x, s->tensors[0].y, kNorm, st));
    for (const Layer& L : s->layers) {
        ConvArgs A{};
        A.in1 = s->tensors[L.in1].y;
        A.in2 = L.in2 >= 0 ? s->tensors[L.in2].y : nullptr;
        A.C1 = L.C1;
        A.C2 = L.C2;
        A.w = s->w16 + L.woff;
        A.bias = s->p + L.boff;
        A.Cout = L.Cout;
        A.N = N;
        A.Din = D >> L.lin;
        A.Dout = D >> L.lout;
        A.mode = L.mode;
        A.out_bf = s->tensors[L.out].y;
        A.act = 1;
        A.slope = kSlope;
        SCHK(launch_conv(A, st));
    }
    const Layer& last = s->layers.back();
    SCHK(launch_head(s->C0, vox, s->tensors[last.out].y, s->p + s->head_w, s->p + s->head_b, s->pred, st));
    return MCRT_OK;
}

mcrt_status backward(mcrt_surrogate* s, int N, int D) {
    hipStream_t st = s->stream;
    const int64_t vox = (int64_t)N * D * D * D;
    SCHK(hipMemsetAsync(s->gp, 0, s->nparam * sizeof(float), st));
    for (size_t i = 1; i < s->tensors.size(); ++i) {
        const Tensor& t = s->tensors[i];
        const int side = D >> t.level;
        SCHK(hipMemsetAsync(t.g, 0, (size_t)N * side * side * side * t.C * sizeof(float), st));
    }
    const Layer& last = s->layers.back();
    SCHK(launch_head_back(s->C0, vox, s->tensors[last.out].y, s->p + s->head_w, s->dpred, s->gp + s->head_w,
                          s->gp + s->head_b, s->tensors[last.out].g, st));
    for (int li = (int)s->layers.size() - 1; li >= 0; --li) {
        const Layer& L = s->layers[li];
        const Tensor& to = s->tensors[L.out];
        const int so = D >> L.lout;
        const int64_t nout = (int64_t)N * so * so * so * L.Cout;
        SCHK(launch_act_back(nout, L.Cout, to.g, to.y, kSlope, 1, s->dz, s->gp + L.boff, st));
        WgradArgs W{};
        W.x1 = s->tensors[L.in1].y;
        W.x2 = L.in2 >= 0 ? s->tensors[L.in2].y : nullptr;
        W.C1 = L.C1;
        W.C2 = L.C2;
        W.dz = s->dz;
        W.Cout = L.Cout;
        W.N = N;
        W.Din = D >> L.lin;
        W.Dout = D >> L.lout;
        W.mode = L.mode;
        W.dw = s->gp + L.woff;
        SCHK(launch_wgrad(W, st));
        if (L.in1 == 0) continue;  // no gradient for the input features
        ConvArgs A{};
        A.in1 = s->dz;
        A.in2 = nullptr;
        A.C1 = L.Cout;
        A.C2 = 0;
        A.w = s->wt16 + L.woff;
        A.bias = nullptr;
        A.Cout = L.C1 + L.C2;
        A.N = N;
        if (L.mode == CONV3) {
            A.mode = CONV3;
            A.Din = A.Dout = D >> L.lout;
        } else if (L.mode == DOWN) {
            A.mode = UP;
            A.Din = D >> L.lout;
            A.Dout = D >> L.lin;
        } else {
            A.mode = DOWN;
            A.Din = D >> L.lout;
            A.Dout = D >> L.lin;
        }
        A.out_f = s->tensors[L.in1].g;
        A.out_f2 = L.in2 >= 0 ? s->tensors[L.in2].g : nullptr;
        A.Csplit = L.C1;
        A.accumulate = 1;
        SCHK(launch_conv(A, st));
    }
    return MCRT_OK;
}

}  // namespace

extern "C" {

mcrt_status mcrt_surrogate_create(mcrt_surrogate** out, int hip_device, int base_channels,
                                  uint64_t seed) {
    if (!out) return MCRT_E_ARG;
    *out = nullptr;
    if (base_channels != 16 && base_channels != 32) return MCRT_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return MCRT_E_DEVICE;
    if (hip_device < 0 || hip_device >= ndev) return MCRT_E_ARG;
    mcrt_surrogate* s = new (std::nothrow) mcrt_surrogate();
    if (!s) return MCRT_E_NOMEM;
    s->device = hip_device;
    s->C0 = base_channels;
    hipSetDevice(hip_device);
    if (hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return MCRT_E_DEVICE;
    }
    s->own_stream = true;
    build_net(s);
    // He-normal weights for LeakyReLU, zero biases, small head
    std::vector<float> h(s->nparam, 0.f);
    std::mt19937_64 rng(seed);
    for (const Layer& L : s->layers) {
        const double fan_in = (double)L.taps * (L.C1 + L.C2);
        std::normal_distribution<double> nd(0.0, sqrt(2.0 / ((1.0 + kSlope * kSlope) * fan_in)));
        for (int64_t i = 0; i < L.nw(); ++i) h[L.woff + i] = (float)nd(rng);
    }
    std::normal_distribution<double> nh(0.0, sqrt(1.0 / s->C0));
    for (int c = 0; c < s->C0; ++c) h[s->head_w + c] = (float)nh(rng);
    h[s->head_b] = 1.5f;  // log10 of a typical dust temperature
    const size_t n = (size_t)s->nparam;
    bool ok = hipMalloc((void**)&s->p, n * 4) == hipSuccess && hipMalloc((void**)&s->gp, n * 4) == hipSuccess &&
              hipMalloc((void**)&s->m1, n * 4) == hipSuccess && hipMalloc((void**)&s->m2, n * 4) == hipSuccess &&
              hipMalloc((void**)&s->w16, n * 2) == hipSuccess && hipMalloc((void**)&s->wt16, n * 2) == hipSuccess &&
              hipMalloc((void**)&s->loss, 2 * sizeof(double)) == hipSuccess;
    if (!ok) {
        mcrt_surrogate_destroy(s);
        return MCRT_E_NOMEM;
    }
    hipMemcpy(s->p, h.data(), n * 4, hipMemcpyHostToDevice);
    hipMemset(s->m1, 0, n * 4);
    hipMemset(s->m2, 0, n * 4);
    hipMemset(s->gp, 0, n * 4);
    if (refresh_bf16(s) != MCRT_OK || hipStreamSynchronize(s->stream) != hipSuccess) {
        mcrt_surrogate_destroy(s);
        return MCRT_E_DEVICE;
    }
    *out = s;
    return MCRT_OK;
}

void mcrt_surrogate_destroy(mcrt_surrogate* s) {
    if (!s) return;
    hipSetDevice(s->device);
    if (s->stream) hipStreamSynchronize(s->stream);
    for (Tensor& t : s->tensors) {
        if (t.y) hipFree(t.y);
        if (t.g) hipFree(t.g);
    }
    float* fb[] = {s->p, s->gp, s->m1, s->m2, s->pred, s->dpred};
    for (float* b : fb)
        if (b) hipFree(b);
    if (s->w16) hipFree(s->w16);
    if (s->wt16) hipFree(s->wt16);
    if (s->dz) hipFree(s->dz);
    if (s->loss) hipFree(s->loss);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    delete s;
}

const char* mcrt_surrogate_last_error(const mcrt_surrogate* s) { return s ? s->err.c_str() : "null"; }

mcrt_status mcrt_surrogate_set_stream(mcrt_surrogate* s, void* hip_stream) {
    if (!s) return MCRT_E_ARG;
    hipSetDevice(s->device);
    hipStreamSynchronize(s->stream);
    if (s->own_stream && s->stream) hipStreamDestroy(s->stream);
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
        s->own_stream = false;
    } else {
        if (hipStreamCreate(&s->stream) != hipSuccess) return sfail(s, MCRT_E_DEVICE, "stream");
        s->own_stream = true;
    }
    return MCRT_OK;
}

int64_t mcrt_surrogate_param_count(const mcrt_surrogate* s) { return s ? s->nparam : -1; }

mcrt_status mcrt_surrogate_set_grad_clip(mcrt_surrogate* s, double max_norm) {
    if (!s) return MCRT_E_ARG;
    if (!(max_norm >= 0.0) || !isfinite(max_norm)) return sfail(s, MCRT_E_ARG, "max_norm must be >= 0");
    s->grad_clip = max_norm;
    return MCRT_OK;
}

mcrt_status mcrt_surrogate_get_params(mcrt_surrogate* s, float* host, size_t n) {
    if (!s || !host) return MCRT_E_ARG;
    if ((int64_t)n != s->nparam) return sfail(s, MCRT_E_SIZE, "parameter count");
    hipSetDevice(s->device);
    SCHK(hipStreamSynchronize(s->stream));
    SCHK(hipMemcpy(host, s->p, n * 4, hipMemcpyDeviceToHost));
    return MCRT_OK;
}

mcrt_status mcrt_surrogate_set_params(mcrt_surrogate* s, const float* host, size_t n) {
    if (!s || !host) return MCRT_E_ARG;
    if ((int64_t)n != s->nparam) return sfail(s, MCRT_E_SIZE, "parameter count");
    for (size_t i = 0; i < n; ++i)
        if (!isfinite(host[i])) return sfail(s, MCRT_E_ARG, "parameters must be finite");
    hipSetDevice(s->device);
    SCHK(hipStreamSynchronize(s->stream));
    SCHK(hipMemcpy(s->p, host, n * 4, hipMemcpyHostToDevice));
    mcrt_status r = refresh_bf16(s);
    if (r != MCRT_OK) return r;
    SCHK(hipStreamSynchronize(s->stream));
    return MCRT_OK;
}

mcrt_status mcrt_surrogate_get_grads(mcrt_surrogate* s, float* host, size_t n) {
    if (!s || !host) return MCRT_E_ARG;
    if ((int64_t)n != s->nparam) return sfail(s, MCRT_E_SIZE, "parameter count");
    hipSetDevice(s->device);
    SCHK(hipStreamSynchronize(s->stream));
    SCHK(hipMemcpy(host, s->gp, n * 4, hipMemcpyDeviceToHost));
    return MCRT_OK;
}

mcrt_status mcrt_surrogate_forward(mcrt_surrogate* s, const float* d_x, int N, int D, float* d_y) {
    if (!s || !d_x || !d_y) return MCRT_E_ARG;
    mcrt_status r = check_shape(s, N, D);
    if (r != MCRT_OK) return r;
    hipSetDevice(s->device);
    r = ensure_buffers(s, N, D, false);
    if (r != MCRT_OK) return r;
    r = forward(s, d_x, N, D);
    if (r != MCRT_OK) return r;
    const int64_t vox = (int64_t)N * D * D * D;
    SCHK(hipMemcpyAsync(d_y, s->pred, vox * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
    SCHK(hipStreamSynchronize(s->stream));
    return MCRT_OK;
}

mcrt_status mcrt_surrogate_train_step(mcrt_surrogate* s, const float* d_x, const float* d_target,
                                      const float* d_mask, int N, int D, double mask_count,
                                      double lr, int apply_update, double* loss) {
    if (!s || !d_x || !d_target || !d_mask) return MCRT_E_ARG;
    mcrt_status r = check_shape(s, N, D);
    if (r != MCRT_OK) return r;
    if (!(mask_count > 0.0) || !(lr >= 0.0)) return sfail(s, MCRT_E_ARG, "mask_count > 0, lr >= 0");
    hipSetDevice(s->device);
    r = ensure_buffers(s, N, D, true);
    if (r != MCRT_OK) return r;
    r = forward(s, d_x, N, D);
    if (r != MCRT_OK) return r;
    const int64_t vox = (int64_t)N * D * D * D;
    SCHK(hipMemsetAsync(s->loss, 0, 2 * sizeof(double), s->stream));
    SCHK(launch_loss(vox, s->pred, d_target, d_mask, (float)(1.0 / mask_count), s->dpred, s->loss,
                     s->stream));
    r = backward(s, N, D);
    if (r != MCRT_OK) return r;
    if (apply_update) {
        s->step++;
        const double b1 = 0.9, b2 = 0.999;
        const double c1 = 1.0 / (1.0 - pow(b1, (double)s->step));
        const double c2 = 1.0 / (1.0 - pow(b2, (double)s->step));
        SCHK(launch_adam(s->nparam, s->p, s->gp, s->m1, s->m2, (float)lr, (float)b1, (float)b2, 1e-8f,
                         (float)c1, (float)c2, (float)s->grad_clip, s->loss + 1, s->stream));
        r = refresh_bf16(s);
        if (r != MCRT_OK) return r;
    }
    double l = 0.0;
    SCHK(hipMemcpyAsync(&l, s->loss, sizeof(double), hipMemcpyDeviceToHost, s->stream));
    SCHK(hipStreamSynchronize(s->stream));
    if (loss) *loss = l / mask_count;
    return MCRT_OK;
}

// log10 T from the network for an N x D^3 batch, written as T into d_T (FP64)
mcrt_status mcrt_surrogate_predict_T(mcrt_surrogate* s, const float* d_x, int N, int D, double* d_T) {
    if (!s || !d_x || !d_T) return MCRT_E_ARG;
    mcrt_status r = check_shape(s, N, D);
    if (r != MCRT_OK) return r;
    hipSetDevice(s->device);
    r = ensure_buffers(s, N, D, false);
    if (r != MCRT_OK) return r;
    r = forward(s, d_x, N, D);
    if (r != MCRT_OK) return r;
    SCHK(launch_exp10((int64_t)N * D * D * D, s->pred, d_T, s->stream));
    SCHK(hipStreamSynchronize(s->stream));
    return MCRT_OK;
}

}  // extern "C"
