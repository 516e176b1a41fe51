// oz_mlp.hip -- the selector network: a 16 -> 64 -> 64 -> 1 perceptron with
// ReLU hidden layers, trained with the pinball (quantile) loss and Adam, all
// in FP32 on the GPU.
//
// Parameter vector (kNParam floats): W1[64][16] (row = hidden unit), b1[64],
// W2[64][64], b2[64], W3[64], b3.  Inputs are normalised, xn = (x - mu) / sd,
// with per-feature mu, sd stored beside the parameters.
//   forward : z1 = W1 xn + b1, h1 = relu(z1), z2 = W2 h1 + b2, h2 = relu(z2),
//             y = W3 . h2 + b3
//   loss    : (1/B) sum_r rho(t_r - y_r), rho(r) = tau r (r > 0), (tau - 1) r
//   Adam    : Kingma and Ba (2015), bias-corrected moments.
// Every sum runs in a fixed order, so results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/oz.h"
#include "oz_handle.h"
#include "oz_internal.h"

namespace {

constexpr uint32_t kMlpMagic = 0x6f7a6d6cu;  // "ozml"
constexpr int kIn = OZ_MLP_NIN, kH = OZ_MLP_NHIDDEN;
constexpr int kW1 = 0, kB1 = kW1 + kH * kIn, kW2 = kB1 + kH, kB2 = kW2 + kH * kH, kW3 = kB2 + kH, kB3 = kW3 + kH;
constexpr int kNParam = kB3 + 1;
static_assert(kNParam == OZ_MLP_NPARAM, "parameter count");
// per-row activations kept by the forward pass for the backward pass
constexpr int kActXn = 0, kActZ1 = kActXn + kIn, kActZ2 = kActZ1 + kH, kActLen = kActZ2 + kH;
constexpr int kRowsPerBlock = 4;  // one wave per row

// ---- forward: one wave per row; lane u owns hidden unit u ------------------
// Weights are staged in LDS transposed (W1T[f][u], W2T[v][u]) so that the 64
// lanes read consecutive words.
__global__ __launch_bounds__(256) void mlp_fwd_kernel(const float* P, const float* mu, const float* sd,
                                                      const float* X, int64_t rows, float* y, float* act) {
    __shared__ float w1t[kIn * kH], w2t[kH * kH], b1[kH], b2[kH], w3[kH];
    __shared__ float xs[kRowsPerBlock][kIn], hs[kRowsPerBlock][kH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kH * kIn; e += 256) w1t[(e % kIn) * kH + e / kIn] = P[kW1 + e];
    for (int e = tid; e < kH * kH; e += 256) w2t[(e % kH) * kH + e / kH] = P[kW2 + e];
    if (tid < kH) {
        b1[tid] = P[kB1 + tid];
        b2[tid] = P[kB2 + tid];
        w3[tid] = P[kW3 + tid];
    }
    const float b3 = P[kB3];
    __syncthreads();
    for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock; r0 < rows;
         r0 += static_cast<int64_t>(gridDim.x) * kRowsPerBlock) {
        const int64_t r = r0 + wave;
        const bool live = r < rows;  // wave-uniform
        if (live && lane < kIn) {
            const float xn = (X[r * kIn + lane] - mu[lane]) / sd[lane];
            xs[wave][lane] = xn;
            if (act) act[r * kActLen + kActXn + lane] = xn;
        }
        __syncthreads();
        float z1 = b1[lane];
        for (int f = 0; f < kIn; ++f) z1 = z1 + w1t[f * kH + lane] * xs[wave][f];
        hs[wave][lane] = z1 > 0.0f ? z1 : 0.0f;
        __syncthreads();
        float z2 = b2[lane];
        for (int v = 0; v < kH; ++v) z2 = z2 + w2t[v * kH + lane] * hs[wave][v];
        float t = w3[lane] * (z2 > 0.0f ? z2 : 0.0f);
        for (int off = 1; off < 64; off <<= 1) t = t + __shfl_xor(t, off);
        if (live) {
            if (act) {
                act[r * kActLen + kActZ1 + lane] = z1;
                act[r * kActLen + kActZ2 + lane] = z2;
            }
            if (lane == 0) y[r] = t + b3;
        }
        __syncthreads();
    }
}

// ---- per-row deltas and loss ---------------------------------------------------
// d3 = dL/dy, d2[u] = d3 W3[u] [z2_u > 0], d1[u] = sum_v W2[v][u] d2[v] [z1_u > 0].
__global__ __launch_bounds__(256) void mlp_delta_kernel(const float* P, const float* t, const float* y,
                                                        const float* act, int64_t rows, float tau, float* d1,
                                                        float* d2, float* d3, float* rowloss) {
    __shared__ float w2[kH * kH], w3[kH];
    __shared__ float ds[kRowsPerBlock][kH];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int e = tid; e < kH * kH; e += 256) w2[e] = P[kW2 + e];
    if (tid < kH) w3[tid] = P[kW3 + tid];
    __syncthreads();
    const float inv_b = 1.0f / static_cast<float>(rows);
    for (int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRowsPerBlock; r0 < rows;
         r0 += static_cast<int64_t>(gridDim.x) * kRowsPerBlock) {
        const int64_t r = r0 + wave;
        const bool live = r < rows;
        float g3 = 0.0f;
        if (live) {
            const float res = t[r] - y[r];
            g3 = (res > 0.0f ? -tau : 1.0f - tau) * inv_b;
            if (lane == 0) {
                d3[r] = g3;
                rowloss[r] = (res > 0.0f ? tau * res : (tau - 1.0f) * res) * inv_b;
            }
        }
        const float z2 = live ? act[r * kActLen + kActZ2 + lane] : 0.0f;
        const float g2 = z2 > 0.0f ? g3 * w3[lane] : 0.0f;
        ds[wave][lane] = g2;
        __syncthreads();
        if (live) {
            d2[r * kH + lane] = g2;
            float g1 = 0.0f;
            for (int v = 0; v < kH; ++v) g1 = g1 + w2[v * kH + lane] * ds[wave][v];
            const float z1 = act[r * kActLen + kActZ1 + lane];
            d1[r * kH + lane] = z1 > 0.0f ? g1 : 0.0f;
        }
        __syncthreads();
    }
}

// ---- parameter gradients: one thread per parameter, rows summed in order -----
__global__ __launch_bounds__(256) void mlp_pgrad_kernel(const float* act, const float* d1, const float* d2,
                                                        const float* d3, int64_t rows, float* grad) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNParam) return;
    float g = 0.0f;
    if (p < kB1) {
        const int u = p / kIn, f = p % kIn;
        for (int64_t r = 0; r < rows; ++r) g = g + d1[r * kH + u] * act[r * kActLen + kActXn + f];
    } else if (p < kW2) {
        const int u = p - kB1;
        for (int64_t r = 0; r < rows; ++r) g = g + d1[r * kH + u];
    } else if (p < kB2) {
        const int u = (p - kW2) / kH, v = (p - kW2) % kH;
        for (int64_t r = 0; r < rows; ++r) {
            const float z1 = act[r * kActLen + kActZ1 + v];
            g = g + d2[r * kH + u] * (z1 > 0.0f ? z1 : 0.0f);
        }
    } else if (p < kW3) {
        const int u = p - kB2;
        for (int64_t r = 0; r < rows; ++r) g = g + d2[r * kH + u];
    } else if (p < kB3) {
        const int u = p - kW3;
        for (int64_t r = 0; r < rows; ++r) {
            const float z2 = act[r * kActLen + kActZ2 + u];
            g = g + d3[r] * (z2 > 0.0f ? z2 : 0.0f);
        }
    } else {
        for (int64_t r = 0; r < rows; ++r) g = g + d3[r];
    }
    grad[p] = g;
}

__global__ void adam_kernel(float* P, const float* g, float* m, float* v, float lr, float b1, float b2, float eps,
                            float bc1, float bc2) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= kNParam) return;
    const float gi = g[p];
    const float mi = b1 * m[p] + (1.0f - b1) * gi;
    const float vi = b2 * v[p] + (1.0f - b2) * gi * gi;
    m[p] = mi;
    v[p] = vi;
    P[p] = P[p] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void gather_kernel(const float* X, const float* t, const int32_t* idx, int64_t rows, float* Xb,
                              float* tb) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (e >= rows * kIn) return;
    const int64_t r = e / kIn, f = e % kIn;
    const int64_t src = idx[r];
    Xb[e] = X[src * kIn + f];
    if (f == 0) tb[r] = t[src];
}

// one block: out[0] = sum of vals in index-strided order, then a fixed tree
__global__ __launch_bounds__(256) void sum_kernel(const float* vals, int64_t n, float* out) {
    __shared__ float red[256];
    float a = 0.0f;
    for (int64_t i = threadIdx.x; i < n; i += 256) a = a + vals[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

__global__ void slices_from_output_kernel(const float* y, int64_t rows, int smin, int smax, int32_t* s) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (r >= rows) return;
    const float v = y[r];
    int q = smax;
    if (v == v) {  // NaN keeps smax
        const float c = floorf(v + 0.5f);
        q = c < static_cast<float>(smin) ? smin : (c > static_cast<float>(smax) ? smax : static_cast<int>(c));
    }
    s[r] = q;
}

}  // namespace

struct oz_mlp_s {
    uint32_t magic;
    oz_handle_t h;
    float* dev;      // params | m | v | grad | mu | sd
    int64_t step;    // Adam steps taken
    // training scratch, sized for cap rows
    int64_t cap;
    float* scratch;  // act | d1 | d2 | d3 | rowloss | y | Xb | tb
    float* P() const { return dev; }
    float* M() const { return dev + kNParam; }
    float* V() const { return dev + 2 * kNParam; }
    float* G() const { return dev + 3 * kNParam; }
    float* mu() const { return dev + 4 * kNParam; }
    float* sd() const { return dev + 4 * kNParam + kIn; }
};

namespace {

constexpr int64_t kDevFloats = 4 * kNParam + 2 * kIn;
constexpr int64_t kRowFloats = kActLen + 2 * kH + 1 + 1 + 1 + kIn + 1;

bool mlp_ok(oz_mlp_t p) { return p != nullptr && p->magic == kMlpMagic; }

int hipst(hipError_t e) { return e == hipSuccess ? OZ_OK : OZ_ERR_HIP; }

int ensure_cap(oz_mlp_t p, int64_t rows) {
    if (rows <= p->cap) return OZ_OK;
    if (p->scratch) {
        hipStreamSynchronize(oz_handle_stream(p->h));
        hipFree(p->scratch);
        p->scratch = nullptr;
        p->cap = 0;
    }
    void* q = nullptr;
    if (hipMalloc(&q, sizeof(float) * kRowFloats * rows) != hipSuccess) return OZ_ERR_ALLOC;
    p->scratch = static_cast<float*>(q);
    p->cap = rows;
    return OZ_OK;
}

struct Scratch {
    float *act, *d1, *d2, *d3, *rowloss, *y, *Xb, *tb;
};
Scratch carve(oz_mlp_t p) {
    Scratch s;
    float* q = p->scratch;
    const int64_t c = p->cap;
    s.act = q;
    q += kActLen * c;
    s.d1 = q;
    q += kH * c;
    s.d2 = q;
    q += kH * c;
    s.d3 = q;
    q += c;
    s.rowloss = q;
    q += c;
    s.y = q;
    q += c;
    s.Xb = q;
    q += kIn * c;
    s.tb = q;
    return s;
}

unsigned fwd_blocks(int64_t rows) {
    const int64_t b = (rows + kRowsPerBlock - 1) / kRowsPerBlock;
    return static_cast<unsigned>(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

hipError_t forward(oz_mlp_t p, int64_t rows, const float* X, float* y, float* act, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3(fwd_blocks(rows)), dim3(256), 0, st, p->P(), p->mu(), p->sd(), X, rows,
                       y, act);
    return hipGetLastError();
}

// gradient of the batch loss into p->G(); loss sum into *loss_dev
hipError_t backward(oz_mlp_t p, int64_t rows, const float* X, const float* t, float tau, float* loss_dev,
                    hipStream_t st) {
    const Scratch s = carve(p);
    hipError_t e = forward(p, rows, X, s.y, s.act, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_delta_kernel, dim3(fwd_blocks(rows)), dim3(256), 0, st, p->P(), t, s.y, s.act, rows, tau,
                       s.d1, s.d2, s.d3, s.rowloss);
    hipLaunchKernelGGL(mlp_pgrad_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, s.act, s.d1, s.d2, s.d3, rows,
                       p->G());
    if (loss_dev) hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, s.rowloss, rows, loss_dev);
    return hipGetLastError();
}

constexpr float kB1m = 0.9f, kB2m = 0.999f, kAdamEps = 1e-8f;

hipError_t adam(oz_mlp_t p, float lr, hipStream_t st) {
    ++p->step;
    const float bc1 = static_cast<float>(1.0 - std::pow(static_cast<double>(kB1m), static_cast<double>(p->step)));
    const float bc2 = static_cast<float>(1.0 - std::pow(static_cast<double>(kB2m), static_cast<double>(p->step)));
    hipLaunchKernelGGL(adam_kernel, dim3((kNParam + 255) / 256), dim3(256), 0, st, p->P(), p->G(), p->M(), p->V(), lr,
                       kB1m, kB2m, kAdamEps, bc1, bc2);
    return hipGetLastError();
}

// He-uniform weights from the splitmix64 stream of `seed`, zero biases.
std::vector<float> init_params(uint64_t seed) {
    std::vector<float> h(kNParam, 0.0f);
    uint64_t c = 0;
    auto uni = [&](double a) {
        const double u = static_cast<double>(oz::sm64_draw(seed, c++) >> 11) * 0x1p-53;
        return static_cast<float>(a * (2.0 * u - 1.0));
    };
    for (int e = 0; e < kH * kIn; ++e) h[kW1 + e] = uni(std::sqrt(6.0 / kIn));
    for (int e = 0; e < kH * kH; ++e) h[kW2 + e] = uni(std::sqrt(6.0 / kH));
    for (int e = 0; e < kH; ++e) h[kW3 + e] = uni(std::sqrt(6.0 / kH));
    return h;
}

const char kFileMagic[8] = {'O', 'Z', 'M', 'L', 'P', '0', '0', '1'};

}  // namespace

hipError_t oz_mlp_predict_device(oz_mlp_t p, int64_t rows, const float* X, float* y, int smin, int smax,
                                 int32_t* s_out, hipStream_t st) {
    hipError_t e = forward(p, rows, X, y, nullptr, st);
    if (e != hipSuccess || rows <= 0) return e;
    hipLaunchKernelGGL(slices_from_output_kernel, dim3(static_cast<unsigned>((rows + 255) / 256)), dim3(256), 0, st,
                       y, rows, smin, smax, s_out);
    return hipGetLastError();
}

bool oz_mlp_valid(oz_mlp_t p) { return mlp_ok(p); }

extern "C" {

int oz_mlp_create(oz_handle_t h, uint64_t seed, oz_mlp_t* out) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (!out) return OZ_ERR_ARG;
    *out = nullptr;
    if (oz_handle_use_device(h)) return OZ_ERR_HIP;
    oz_mlp_s* p = new (std::nothrow) oz_mlp_s;
    if (!p) return OZ_ERR_ALLOC;
    p->magic = kMlpMagic;
    p->h = h;
    p->step = 0;
    p->cap = 0;
    p->scratch = nullptr;
    void* d = nullptr;
    if (hipMalloc(&d, sizeof(float) * kDevFloats) != hipSuccess) {
        delete p;
        return OZ_ERR_ALLOC;
    }
    p->dev = static_cast<float*>(d);
    std::vector<float> host(kDevFloats, 0.0f);
    const std::vector<float> w = init_params(seed);
    std::memcpy(host.data(), w.data(), sizeof(float) * kNParam);
    for (int f = 0; f < kIn; ++f) host[4 * kNParam + kIn + f] = 1.0f;  // sd = 1
    if (hipMemcpy(p->dev, host.data(), sizeof(float) * kDevFloats, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(p->dev);
        delete p;
        return OZ_ERR_HIP;
    }
    *out = p;
    return OZ_OK;
}

int oz_mlp_destroy(oz_mlp_t p) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (oz_handle_valid(p->h)) {
        oz_handle_use_device(p->h);
        hipStreamSynchronize(oz_handle_stream(p->h));
        if (oz_handle_selector(p->h) == p) oz_handle_set_selector(p->h, nullptr);
    }
    hipFree(p->dev);
    if (p->scratch) hipFree(p->scratch);
    p->magic = 0;
    delete p;
    return OZ_OK;
}

int oz_mlp_set_params(oz_mlp_t p, const float* params, const float* mu, const float* sd) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    hipStream_t st = oz_handle_stream(p->h);
    if (hipStreamSynchronize(st) != hipSuccess) return OZ_ERR_HIP;
    if (sd)
        for (int f = 0; f < kIn; ++f)
            if (!(sd[f] > 0.0f)) return OZ_ERR_ARG;
    hipError_t e = hipSuccess;
    if (params) {
        e = hipMemcpy(p->P(), params, sizeof(float) * kNParam, hipMemcpyHostToDevice);
        // a new parameter vector restarts the optimiser
        if (e == hipSuccess) e = hipMemset(p->M(), 0, sizeof(float) * 2 * kNParam);
        p->step = 0;
    }
    if (e == hipSuccess && mu) e = hipMemcpy(p->mu(), mu, sizeof(float) * kIn, hipMemcpyHostToDevice);
    if (e == hipSuccess && sd) e = hipMemcpy(p->sd(), sd, sizeof(float) * kIn, hipMemcpyHostToDevice);
    return hipst(e);
}

int oz_mlp_get_params(oz_mlp_t p, float* params, float* mu, float* sd) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    if (hipStreamSynchronize(oz_handle_stream(p->h)) != hipSuccess) return OZ_ERR_HIP;
    hipError_t e = hipSuccess;
    if (params) e = hipMemcpy(params, p->P(), sizeof(float) * kNParam, hipMemcpyDeviceToHost);
    if (e == hipSuccess && mu) e = hipMemcpy(mu, p->mu(), sizeof(float) * kIn, hipMemcpyDeviceToHost);
    if (e == hipSuccess && sd) e = hipMemcpy(sd, p->sd(), sizeof(float) * kIn, hipMemcpyDeviceToHost);
    return hipst(e);
}

int oz_mlp_fit_norm(oz_mlp_t p, int64_t rows, const float* X) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (rows <= 0 || !X) return OZ_ERR_ARG;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    if (hipStreamSynchronize(oz_handle_stream(p->h)) != hipSuccess) return OZ_ERR_HIP;
    std::vector<float> host(static_cast<size_t>(rows) * kIn);
    if (hipMemcpy(host.data(), X, sizeof(float) * host.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return OZ_ERR_HIP;
    float mu[kIn], sd[kIn];
    for (int f = 0; f < kIn; ++f) {
        double s = 0.0;
        for (int64_t r = 0; r < rows; ++r) s += host[r * kIn + f];
        const double mean = s / static_cast<double>(rows);
        double q = 0.0;
        for (int64_t r = 0; r < rows; ++r) {
            const double d = host[r * kIn + f] - mean;
            q += d * d;
        }
        const double sdev = std::sqrt(q / static_cast<double>(rows));
        mu[f] = static_cast<float>(mean);
        sd[f] = static_cast<float>(sdev > 1e-6 ? sdev : 1.0);
    }
    return oz_mlp_set_params(p, nullptr, mu, sd);
}

int oz_mlp_forward(oz_mlp_t p, int64_t rows, const float* X, float* y) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (rows < 0 || (rows > 0 && (!X || !y))) return OZ_ERR_ARG;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    return hipst(forward(p, rows, X, y, nullptr, oz_handle_stream(p->h)));
}

int oz_mlp_grad(oz_mlp_t p, int64_t rows, const float* X, const float* t, float tau, float* grad, float* loss) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (rows <= 0 || !X || !t || !(tau > 0.0f && tau < 1.0f)) return OZ_ERR_ARG;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    int st = ensure_cap(p, rows);
    if (st) return st;
    hipStream_t s = oz_handle_stream(p->h);
    const Scratch sc = carve(p);
    if (backward(p, rows, X, t, tau, sc.tb, s) != hipSuccess) return OZ_ERR_HIP;
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && grad) e = hipMemcpy(grad, p->G(), sizeof(float) * kNParam, hipMemcpyDeviceToHost);
    if (e == hipSuccess && loss) e = hipMemcpy(loss, sc.tb, sizeof(float), hipMemcpyDeviceToHost);
    return hipst(e);
}

int oz_mlp_train_step(oz_mlp_t p, int64_t rows, const float* X, const float* t, float tau, float lr, float* loss) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (rows <= 0 || !X || !t || !(tau > 0.0f && tau < 1.0f) || !(lr > 0.0f)) return OZ_ERR_ARG;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    int st = ensure_cap(p, rows);
    if (st) return st;
    hipStream_t s = oz_handle_stream(p->h);
    const Scratch sc = carve(p);
    if (backward(p, rows, X, t, tau, sc.tb, s) != hipSuccess || adam(p, lr, s) != hipSuccess) return OZ_ERR_HIP;
    if (!loss) return OZ_OK;
    if (hipStreamSynchronize(s) != hipSuccess) return OZ_ERR_HIP;
    return hipst(hipMemcpy(loss, sc.tb, sizeof(float), hipMemcpyDeviceToHost));
}

int oz_mlp_train(oz_mlp_t p, int64_t rows, const float* X, const float* t, int32_t epochs, int32_t batch, float tau,
                 float lr, uint64_t seed, float* epoch_loss) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (rows <= 0 || !X || !t || epochs < 1 || batch < 1 || !(tau > 0.0f && tau < 1.0f) || !(lr > 0.0f))
        return OZ_ERR_ARG;
    if (rows > INT32_MAX) return OZ_ERR_ARG;
    if (oz_handle_use_device(p->h)) return OZ_ERR_HIP;
    const int64_t B = batch < rows ? batch : rows;
    int st = ensure_cap(p, B);
    if (st) return st;
    hipStream_t s = oz_handle_stream(p->h);
    const int64_t nb = (rows + B - 1) / B;
    void *idx_dev = nullptr, *loss_dev = nullptr;
    if (hipMalloc(&idx_dev, sizeof(int32_t) * rows) != hipSuccess) return OZ_ERR_ALLOC;
    if (hipMalloc(&loss_dev, sizeof(float) * nb) != hipSuccess) {
        hipFree(idx_dev);
        return OZ_ERR_ALLOC;
    }
    // a fresh network starts its output at the mean target
    if (p->step == 0) {
        std::vector<float> th(static_cast<size_t>(rows));
        if (hipStreamSynchronize(s) != hipSuccess ||
            hipMemcpy(th.data(), t, sizeof(float) * rows, hipMemcpyDeviceToHost) != hipSuccess) {
            hipFree(idx_dev);
            hipFree(loss_dev);
            return OZ_ERR_HIP;
        }
        double sum = 0.0;
        for (float v : th) sum += v;
        const float b3 = static_cast<float>(sum / static_cast<double>(rows));
        if (hipMemcpy(p->P() + kB3, &b3, sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            hipFree(idx_dev);
            hipFree(loss_dev);
            return OZ_ERR_HIP;
        }
    }
    const Scratch sc = carve(p);
    std::vector<int32_t> perm(static_cast<size_t>(rows));
    std::vector<float> lh(static_cast<size_t>(nb));
    hipError_t e = hipSuccess;
    uint64_t ctr = 0;
    for (int32_t ep = 0; ep < epochs && e == hipSuccess; ++ep) {
        // Fisher-Yates shuffle driven by the splitmix64 stream of `seed`
        for (int64_t r = 0; r < rows; ++r) perm[r] = static_cast<int32_t>(r);
        for (int64_t r = rows - 1; r > 0; --r) {
            const uint64_t j = oz::sm64_draw(seed, ctr++) % static_cast<uint64_t>(r + 1);
            std::swap(perm[r], perm[j]);
        }
        e = hipMemcpyAsync(idx_dev, perm.data(), sizeof(int32_t) * rows, hipMemcpyHostToDevice, s);
        for (int64_t b = 0; b < nb && e == hipSuccess; ++b) {
            const int64_t r0 = b * B, nr = (r0 + B <= rows) ? B : rows - r0;
            hipLaunchKernelGGL(gather_kernel, dim3(static_cast<unsigned>((nr * kIn + 255) / 256)), dim3(256), 0, s, X,
                               t, static_cast<const int32_t*>(idx_dev) + r0, nr, sc.Xb, sc.tb);
            e = backward(p, nr, sc.Xb, sc.tb, tau, static_cast<float*>(loss_dev) + b, s);
            if (e == hipSuccess) e = adam(p, lr, s);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);  // perm is rewritten next epoch
        if (e == hipSuccess && epoch_loss) {
            e = hipMemcpy(lh.data(), loss_dev, sizeof(float) * nb, hipMemcpyDeviceToHost);
            // per-batch mean losses, weighted by batch size
            double tot = 0.0;
            for (int64_t b = 0; b < nb; ++b) {
                const int64_t nr = (b * B + B <= rows) ? B : rows - b * B;
                tot += static_cast<double>(lh[b]) * static_cast<double>(nr);
            }
            epoch_loss[ep] = static_cast<float>(tot / static_cast<double>(rows));
        }
    }
    hipFree(idx_dev);
    hipFree(loss_dev);
    return hipst(e);
}

int oz_mlp_save(oz_mlp_t p, const char* path) {
    if (!mlp_ok(p)) return OZ_ERR_HANDLE;
    if (!path) return OZ_ERR_ARG;
    std::vector<float> w(kNParam + 2 * kIn);
    int st = oz_mlp_get_params(p, w.data(), w.data() + kNParam, w.data() + kNParam + kIn);
    if (st) return st;
    FILE* f = std::fopen(path, "wb");
    if (!f) return OZ_ERR_ARG;
    const int32_t dims[3] = {kIn, kH, kNParam};
    bool ok = std::fwrite(kFileMagic, 1, 8, f) == 8 && std::fwrite(dims, sizeof(int32_t), 3, f) == 3 &&
              std::fwrite(w.data(), sizeof(float), w.size(), f) == w.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? OZ_OK : OZ_ERR_ARG;
}

int oz_mlp_load(oz_handle_t h, const char* path, oz_mlp_t* out) {
    if (!oz_handle_valid(h)) return OZ_ERR_HANDLE;
    if (!path || !out) return OZ_ERR_ARG;
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return OZ_ERR_ARG;
    char magic[8];
    int32_t dims[3];
    std::vector<float> w(kNParam + 2 * kIn);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kFileMagic, 8) == 0 &&
              std::fread(dims, sizeof(int32_t), 3, f) == 3 && dims[0] == kIn && dims[1] == kH &&
              dims[2] == kNParam && std::fread(w.data(), sizeof(float), w.size(), f) == w.size();
    std::fclose(f);
    if (!ok) return OZ_ERR_ARG;
    oz_mlp_t p = nullptr;
    int st = oz_mlp_create(h, 0, &p);
    if (st) return st;
    st = oz_mlp_set_params(p, w.data(), w.data() + kNParam, w.data() + kNParam + kIn);
    if (st) {
        oz_mlp_destroy(p);
        return st;
    }
    *out = p;
    return OZ_OK;
}

}  // extern "C"
