// K9 / K10: the learned format-and-kernel selector (the paper's offline data
// mining model of Section 5, Equation 1, here a 12-64-64-C perceptron) --
// inference on raw features, and the forward, backward and Adam kernels that
// train it.  float32 throughout; every reduction runs in a fixed order, so
// results are deterministic.
//
// Parameter order (flat float32): W1 [64 x 12], b1 [64], W2 [64 x 64],
// b2 [64], W3 [C x 64], b3 [C], row-major.
#include "internal.hpp"

namespace smat {
namespace {

constexpr int kIn = 12;
constexpr int kHid = 64;

struct Net {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
};

__host__ __device__ inline Net unpack(const float *p, int n_out) {
    Net n;
    n.W1 = p;
    n.b1 = n.W1 + kHid * kIn;
    n.W2 = n.b1 + kHid;
    n.b2 = n.W2 + kHid * kHid;
    n.W3 = n.b2 + kHid;
    n.b3 = n.W3 + n_out * kHid;
    return n;
}

__device__ __forceinline__ bool is_log_feature(int j) { return j <= 5 || j == 9; }

// One workgroup of 64 threads per feature row.
__global__ __launch_bounds__(64) void k_mlp_infer(const float *__restrict__ params, int n_out,
                                                  const float *__restrict__ mean,
                                                  const float *__restrict__ stdv,
                                                  const float *__restrict__ raw,
                                                  float *__restrict__ scores) {
    __shared__ float z[kIn];
    __shared__ float h1[kHid];
    __shared__ float h2[kHid];
    const Net net = unpack(params, n_out);
    const int t = threadIdx.x;
    const int64_t row = blockIdx.x;
    if (t < kIn) {
        float g = raw[row * kIn + t];
        if (is_log_feature(t)) g = log1pf(fmaxf(g, 0.0f));
        z[t] = (g - mean[t]) / stdv[t];
    }
    __syncthreads();
    float a = net.b1[t];
    for (int k = 0; k < kIn; ++k) a = fmaf(net.W1[t * kIn + k], z[k], a);
    h1[t] = fmaxf(a, 0.0f);
    __syncthreads();
    a = net.b2[t];
    for (int k = 0; k < kHid; ++k) a = fmaf(net.W2[t * kHid + k], h1[k], a);
    h2[t] = fmaxf(a, 0.0f);
    __syncthreads();
    if (t < n_out) {
        a = net.b3[t];
        for (int k = 0; k < kHid; ++k) a = fmaf(net.W3[t * kHid + k], h2[k], a);
        scores[row * n_out + t] = a;
    }
}

// out[b, j] = act(sum_k W[j, k] in[b, k] + bias[j]); one thread per (b, j).
__global__ void k_dense(const float *__restrict__ in, const float *__restrict__ W,
                        const float *__restrict__ bias, float *__restrict__ out, int64_t B,
                        int nin, int nout, int relu) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * nout) return;
    int64_t b = t / nout;
    int j = (int)(t % nout);
    float a = bias[j];
    for (int k = 0; k < nin; ++k) a = fmaf(W[j * nin + k], in[b * nin + k], a);
    out[t] = relu ? fmaxf(a, 0.0f) : a;
}

// loss = sum mask (s - t)^2 / max(1, sum mask); ds = 2 mask (s - t) / cnt.
// One workgroup of 256 threads, fixed-order partial sums.
__global__ __launch_bounds__(256) void k_loss_grad(const float *__restrict__ s,
                                                   const float *__restrict__ target,
                                                   const float *__restrict__ mask, int64_t count,
                                                   float *__restrict__ ds, float *__restrict__ loss) {
    __shared__ float red[256];
    __shared__ float red2[256];
    float c = 0.0f, l = 0.0f;
    for (int64_t i = threadIdx.x; i < count; i += 256) {
        float mk = mask[i];
        if (mk > 0.0f) {
            float r = s[i] - target[i];
            c += 1.0f;
            l = fmaf(r, r, l);
        }
    }
    red[threadIdx.x] = c;
    red2[threadIdx.x] = l;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            red[threadIdx.x] += red[threadIdx.x + off];
            red2[threadIdx.x] += red2[threadIdx.x + off];
        }
        __syncthreads();
    }
    const float cnt = fmaxf(red[0], 1.0f);
    if (threadIdx.x == 0) *loss = red2[0] / cnt;
    for (int64_t i = threadIdx.x; i < count; i += 256)
        ds[i] = mask[i] > 0.0f ? 2.0f * (s[i] - target[i]) / cnt : 0.0f;
}

// din[b, k] = (sum_j dout[b, j] W[j, k]) * (act[b, k] > 0)
__global__ void k_backprop_input(const float *__restrict__ dout, const float *__restrict__ W,
                                 const float *__restrict__ act, float *__restrict__ din, int64_t B,
                                 int nin, int nout) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= B * nin) return;
    int64_t b = t / nin;
    int k = (int)(t % nin);
    float a = 0.0f;
    for (int j = 0; j < nout; ++j) a = fmaf(dout[b * nout + j], W[j * nin + k], a);
    din[t] = act[t] > 0.0f ? a : 0.0f;
}

// gW[j, k] = sum_b dout[b, j] in[b, k]; gb[j] = sum_b dout[b, j].
// Threads [0, nout*nin) do weights, the next nout threads the biases.
__global__ void k_weight_grad(const float *__restrict__ dout, const float *__restrict__ in,
                              float *__restrict__ gW, float *__restrict__ gb, int64_t B, int nin,
                              int nout) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t nw = (int64_t)nout * nin;
    if (t < nw) {
        int j = (int)(t / nin), k = (int)(t % nin);
        float a = 0.0f;
        for (int64_t b = 0; b < B; ++b) a = fmaf(dout[b * nout + j], in[b * nin + k], a);
        gW[t] = a;
    } else if (t < nw + nout) {
        int j = (int)(t - nw);
        float a = 0.0f;
        for (int64_t b = 0; b < B; ++b) a += dout[b * nout + j];
        gb[j] = a;
    }
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float beta1, float beta2,
                       float eps, float c1, float c2) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = beta1 * m[i] + (1.0f - beta1) * gi;
    float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float mhat = mi / c1, vhat = vi / c2;
    p[i] -= lr * mhat / (sqrtf(vhat) + eps);
}

inline unsigned blocks(int64_t work, int bs) { return (unsigned)((work + bs - 1) / bs); }

struct Work {
    float *h1, *h2, *ds, *dh2, *dh1;
};

inline Work carve(float *ws, int64_t B, int n_out) {
    Work w;
    w.h1 = ws;
    w.h2 = w.h1 + B * kHid;
    w.ds = w.h2 + B * kHid;
    w.dh2 = w.ds + B * n_out;
    w.dh1 = w.dh2 + B * kHid;
    return w;
}

spmv_status forward_into(const float *params, int n_out, const float *x, int64_t B,
                         float *scores, const Work &w, hipStream_t s) {
    Net net = unpack(params, n_out);
    k_dense<<<blocks(B * kHid, 256), 256, 0, s>>>(x, net.W1, net.b1, w.h1, B, kIn, kHid, 1);
    k_dense<<<blocks(B * kHid, 256), 256, 0, s>>>(w.h1, net.W2, net.b2, w.h2, B, kHid, kHid, 1);
    k_dense<<<blocks(B * n_out, 256), 256, 0, s>>>(w.h2, net.W3, net.b3, scores, B, kHid, n_out,
                                                   0);
    SMAT_LAUNCHED("mlp_forward");
    return SPMV_OK;
}

}  // namespace

spmv_status run_mlp_infer(const float *params, int n_out, const float *mean, const float *stdv,
                          const float *raw, int64_t rows, float *scores, hipStream_t s) {
    if (rows == 0) return SPMV_OK;
    k_mlp_infer<<<(unsigned)rows, 64, 0, s>>>(params, n_out, mean, stdv, raw, scores);
    SMAT_LAUNCHED("mlp_infer");
    return SPMV_OK;
}

}  // namespace smat

using namespace smat;

extern "C" int64_t spmv_mlp_param_count(int32_t n_out) {
    return (int64_t)kHid * kIn + kHid + (int64_t)kHid * kHid + kHid + (int64_t)n_out * kHid + n_out;
}

extern "C" int64_t spmv_mlp_workspace_floats(int64_t batch) {
    return batch * (4 * kHid + 2 * SPMV_K_COUNT) + 64;
}

extern "C" spmv_status spmv_mlp_forward(const float *params_dev, int32_t n_out, const float *x_dev,
                                        int64_t batch, float *scores_dev, float *workspace_dev,
                                        void *stream) {
    if (!params_dev || !x_dev || !scores_dev || !workspace_dev || batch < 0 || n_out <= 0 ||
        n_out > SPMV_K_COUNT) {
        set_error("spmv_mlp_forward: bad argument");
        return SPMV_EINVAL;
    }
    if (batch == 0) return SPMV_OK;
    return forward_into(params_dev, n_out, x_dev, batch, scores_dev,
                        carve(workspace_dev, batch, n_out), (hipStream_t)stream);
}

extern "C" spmv_status spmv_mlp_backward(const float *params_dev, int32_t n_out, const float *x_dev,
                                         const float *target_dev, const float *mask_dev,
                                         int64_t batch, float *grad_dev, float *loss_dev,
                                         float *workspace_dev, void *stream) {
    if (!params_dev || !x_dev || !target_dev || !mask_dev || !grad_dev || !loss_dev ||
        !workspace_dev || batch <= 0 || n_out <= 0 || n_out > SPMV_K_COUNT) {
        set_error("spmv_mlp_backward: bad argument");
        return SPMV_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    Work w = carve(workspace_dev, batch, n_out);
    // scores go to the tail of the workspace (after dh1)
    float *scores = w.dh1 + batch * kHid;
    spmv_status st = forward_into(params_dev, n_out, x_dev, batch, scores, w, s);
    if (st != SPMV_OK) return st;
    Net net = unpack(params_dev, n_out);
    Net g = unpack(grad_dev, n_out);
    k_loss_grad<<<1, 256, 0, s>>>(scores, target_dev, mask_dev, batch * n_out, w.ds, loss_dev);
    k_weight_grad<<<blocks((int64_t)n_out * kHid + n_out, 256), 256, 0, s>>>(
        w.ds, w.h2, (float *)g.W3, (float *)g.b3, batch, kHid, n_out);
    k_backprop_input<<<blocks(batch * kHid, 256), 256, 0, s>>>(w.ds, net.W3, w.h2, w.dh2, batch,
                                                               kHid, n_out);
    k_weight_grad<<<blocks((int64_t)kHid * kHid + kHid, 256), 256, 0, s>>>(
        w.dh2, w.h1, (float *)g.W2, (float *)g.b2, batch, kHid, kHid);
    k_backprop_input<<<blocks(batch * kHid, 256), 256, 0, s>>>(w.dh2, net.W2, w.h1, w.dh1, batch,
                                                               kHid, kHid);
    k_weight_grad<<<blocks((int64_t)kHid * kIn + kHid, 256), 256, 0, s>>>(
        w.dh1, x_dev, (float *)g.W1, (float *)g.b1, batch, kIn, kHid);
    SMAT_LAUNCHED("mlp_backward");
    return SPMV_OK;
}

extern "C" spmv_status spmv_mlp_adam(float *params_dev, const float *grad_dev, float *adam_m_dev,
                                     float *adam_v_dev, int64_t n_params, int32_t step, float lr,
                                     float beta1, float beta2, float eps, void *stream) {
    if (!params_dev || !grad_dev || !adam_m_dev || !adam_v_dev || n_params < 0 || step < 1) {
        set_error("spmv_mlp_adam: bad argument");
        return SPMV_EINVAL;
    }
    if (n_params == 0) return SPMV_OK;
    float c1 = (float)(1.0 - pow((double)beta1, (double)step));
    float c2 = (float)(1.0 - pow((double)beta2, (double)step));
    k_adam<<<blocks(n_params, 256), 256, 0, (hipStream_t)stream>>>(
        params_dev, grad_dev, adam_m_dev, adam_v_dev, n_params, lr, beta1, beta2, eps, c1, c2);
    SMAT_LAUNCHED("mlp_adam");
    return SPMV_OK;
}
