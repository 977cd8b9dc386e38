// Precision-selector MLP (16 -> 64 -> 64 -> 3, ReLU, softmax, mean
// cross-entropy, Adam) in binary32.
//
// Parameter blob (5443 floats): W1 (64x16, row-major W1[o][i]), b1 (64),
// W2 (64x64), b2 (64), W3 (3x64), b3 (3).
//
// Forward: one thread per sample, weights staged in LDS.
// Training step (deterministic): each workgroup takes 64 samples, keeps their
// activations and back-propagated signals in LDS, and forms its partial
// gradient with one thread per parameter summing over its samples in a fixed
// order; a second kernel sums the partials in workgroup order, divides by
// the batch size and applies Adam (Kingma & Ba, Algorithm 1).
#include <algorithm>
#include "common.hpp"
#include "kernels.hpp"
#include "../../include/sylv.h"

namespace sylv {

constexpr int NIN = 16, NH = 64, NOUT = 3;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH, NPAR = OB3 + NOUT;
static_assert(NPAR == 5443, "parameter count");
constexpr int SPB = 64;  // samples per workgroup in training

__global__ __launch_bounds__(256) void k_mlp_forward(int n, const float *__restrict__ X,
                                                     const float *__restrict__ P,
                                                     float *__restrict__ probs) {
    __shared__ float w[NPAR];
    for (int e = threadIdx.x; e < NPAR; e += 256) w[e] = P[e];
    __syncthreads();
    const int s = blockIdx.x * 256 + threadIdx.x;
    if (s >= n) return;
    float x[NIN], h1[NH];
    for (int i = 0; i < NIN; ++i) x[i] = X[(size_t)s * NIN + i];
    for (int o = 0; o < NH; ++o) {
        float a = w[OB1 + o];
        for (int i = 0; i < NIN; ++i) a += w[OW1 + o * NIN + i] * x[i];
        h1[o] = a > 0.f ? a : 0.f;
    }
    float z3[NOUT];
    for (int k = 0; k < NOUT; ++k) z3[k] = w[OB3 + k];
    for (int o = 0; o < NH; ++o) {
        float a = w[OB2 + o];
        for (int i = 0; i < NH; ++i) a += w[OW2 + o * NH + i] * h1[i];
        float h2 = a > 0.f ? a : 0.f;
        for (int k = 0; k < NOUT; ++k) z3[k] += w[OW3 + k * NH + o] * h2;
    }
    float mx = fmaxf(z3[0], fmaxf(z3[1], z3[2]));
    float e0 = expf(z3[0] - mx), e1 = expf(z3[1] - mx), e2 = expf(z3[2] - mx);
    float inv = 1.f / (e0 + e1 + e2);
    probs[(size_t)s * 3 + 0] = e0 * inv;
    probs[(size_t)s * 3 + 1] = e1 * inv;
    probs[(size_t)s * 3 + 2] = e2 * inv;
}

// partial gradients: part[blk][NPAR]; losses per sample -> lossv[s]
__global__ __launch_bounds__(256) void k_mlp_grad(int n, const float *__restrict__ X,
                                                  const int *__restrict__ y,
                                                  const float *__restrict__ P,
                                                  float *__restrict__ part, float *__restrict__ lossv) {
    __shared__ float w[NPAR];
    __shared__ float sx[SPB][NIN];
    __shared__ float sh1[SPB][NH];
    __shared__ float sh2[SPB][NH];
    __shared__ float sg1[SPB][NH];
    __shared__ float sg2[SPB][NH];
    __shared__ float sg3[SPB][4];
    for (int e = threadIdx.x; e < NPAR; e += 256) w[e] = P[e];
    const int s0 = blockIdx.x * SPB;
    const int cnt = (n - s0) < SPB ? (n - s0) : SPB;
    for (int e = threadIdx.x; e < SPB * NIN; e += 256) {
        int s = e / NIN, i = e % NIN;
        sx[s][i] = (s < cnt) ? X[(size_t)(s0 + s) * NIN + i] : 0.f;
    }
    __syncthreads();
    // layer 1 (sample, unit) pairs
    for (int e = threadIdx.x; e < SPB * NH; e += 256) {
        int s = e / NH, o = e % NH;
        float a = w[OB1 + o];
        for (int i = 0; i < NIN; ++i) a += w[OW1 + o * NIN + i] * sx[s][i];
        sh1[s][o] = a;  // pre-activation kept for the ReLU mask
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SPB * NH; e += 256) {
        int s = e / NH, o = e % NH;
        float a = w[OB2 + o];
        for (int i = 0; i < NH; ++i) a += w[OW2 + o * NH + i] * fmaxf(sh1[s][i], 0.f);
        sh2[s][o] = a;
    }
    __syncthreads();
    if (threadIdx.x < SPB) {
        int s = threadIdx.x;
        float z[NOUT];
        for (int k = 0; k < NOUT; ++k) {
            float a = w[OB3 + k];
            for (int i = 0; i < NH; ++i) a += w[OW3 + k * NH + i] * fmaxf(sh2[s][i], 0.f);
            z[k] = a;
        }
        float mx = fmaxf(z[0], fmaxf(z[1], z[2]));
        float e0 = expf(z[0] - mx), e1 = expf(z[1] - mx), e2 = expf(z[2] - mx);
        float sum = e0 + e1 + e2;
        float p[3] = {e0 / sum, e1 / sum, e2 / sum};
        if (s < cnt) {
            int lab = y[s0 + s];
            lossv[s0 + s] = -(z[lab] - mx - logf(sum));
            for (int k = 0; k < NOUT; ++k) sg3[s][k] = p[k] - (k == lab ? 1.f : 0.f);
        } else {
            for (int k = 0; k < NOUT; ++k) sg3[s][k] = 0.f;
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SPB * NH; e += 256) {
        int s = e / NH, o = e % NH;
        float g = 0.f;
        for (int k = 0; k < NOUT; ++k) g += w[OW3 + k * NH + o] * sg3[s][k];
        sg2[s][o] = (sh2[s][o] > 0.f) ? g : 0.f;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SPB * NH; e += 256) {
        int s = e / NH, o = e % NH;
        float g = 0.f;
        for (int k = 0; k < NH; ++k) g += w[OW2 + k * NH + o] * sg2[s][k];
        sg1[s][o] = (sh1[s][o] > 0.f) ? g : 0.f;
    }
    __syncthreads();
    float *out = part + (size_t)blockIdx.x * NPAR;
    for (int q = threadIdx.x; q < NPAR; q += 256) {
        float acc = 0.f;
        if (q < OB1) { int o = q / NIN, i = q % NIN; for (int s = 0; s < SPB; ++s) acc += sg1[s][o] * sx[s][i]; }
        else if (q < OW2) { int o = q - OB1; for (int s = 0; s < SPB; ++s) acc += sg1[s][o]; }
        else if (q < OB2) { int o = (q - OW2) / NH, i = (q - OW2) % NH; for (int s = 0; s < SPB; ++s) acc += sg2[s][o] * fmaxf(sh1[s][i], 0.f); }
        else if (q < OW3) { int o = q - OB2; for (int s = 0; s < SPB; ++s) acc += sg2[s][o]; }
        else if (q < OB3) { int k = (q - OW3) / NH, i = (q - OW3) % NH; for (int s = 0; s < SPB; ++s) acc += sg3[s][k] * fmaxf(sh2[s][i], 0.f); }
        else { int k = q - OB3; for (int s = 0; s < SPB; ++s) acc += sg3[s][k]; }
        out[q] = acc;
    }
}

__global__ __launch_bounds__(256) void k_mlp_adam(int n, int nblk, const float *__restrict__ part,
                                                  float *__restrict__ P, float *__restrict__ m,
                                                  float *__restrict__ v, int t, float lr,
                                                  float *__restrict__ grad) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= NPAR) return;
    float g = 0.f;
    for (int b = 0; b < nblk; ++b) g += part[(size_t)b * NPAR + q];
    g /= (float)n;
    if (grad) grad[q] = g;
    // beta1 = 0.9, beta2 = 0.999 (Kingma & Ba); 1 - beta is written as its
    // own constant (1.f - 0.999f is 1.3e-5 away from 0.001 in binary32) and
    // the bias corrections are formed in binary64
    const float b1 = 0.9f, b2 = 0.999f, omb1 = 0.1f, omb2 = 0.001f, eps = 1e-8f;
    float mq = b1 * m[q] + omb1 * g;
    float vq = b2 * v[q] + omb2 * g * g;
    m[q] = mq;
    v[q] = vq;
    const float c1 = (float)(1.0 - pow(0.9, (double)t)), c2 = (float)(1.0 - pow(0.999, (double)t));
    float mh = mq / c1;
    float vh = vq / c2;
    P[q] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ void k_sum_loss(int n, const float *lossv, float *out) {
    __shared__ float red[256];
    float a = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) a += lossv[i];
    red[threadIdx.x] = a;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] / (float)n;
}

// Per-feature mean and standard deviation (population, binary64 sums in a
// fixed order) of n raw feature rows; a deviation below 1e-6 is set to 1.
__global__ __launch_bounds__(256) void k_feat_stats(int n, const float *__restrict__ F, float *mean, float *sd) {
    __shared__ double r1[256], r2[256];
    const int k = blockIdx.x;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double v = F[(size_t)i * NIN + k];
        a += v;
        b += v * v;
    }
    r1[threadIdx.x] = a;
    r2[threadIdx.x] = b;
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if (threadIdx.x < st) {
            r1[threadIdx.x] += r1[threadIdx.x + st];
            r2[threadIdx.x] += r2[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double mu = r1[0] / n;
        const double var = fmax(r2[0] / n - mu * mu, 0.0);
        const double d = sqrt(var);
        mean[k] = (float)mu;
        sd[k] = d < 1e-6 ? 1.f : (float)d;
    }
}

// Z = (F - mean) / sd, row-major n x 16
__global__ void k_standardize(int n, const float *__restrict__ F, const float *__restrict__ mean,
                              const float *__restrict__ sd, float *__restrict__ Z) {
    const size_t total = (size_t)n * NIN;
    for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e % NIN);
        const float d = sd[k] > 0.f ? sd[k] : 1.f;
        Z[e] = (F[e] - mean[k]) / d;
    }
}

// rows perm[0..cnt) of Z and labels into Zb, yb
__global__ void k_gather_rows(int cnt, const int *__restrict__ perm, const float *__restrict__ Z,
                              const int *__restrict__ y, float *__restrict__ Zb, int *__restrict__ yb) {
    const int total = cnt * NIN;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int r = e / NIN, k = e % NIN;
        const int src = perm[r];
        Zb[e] = Z[(size_t)src * NIN + k];
        if (k == 0) yb[r] = y[src];
    }
}

void mlp_feature_stats(hipStream_t s, int n, const float *F, float *mean, float *sd) {
    hipLaunchKernelGGL(k_feat_stats, dim3(NIN), dim3(256), 0, s, n, F, mean, sd);
}
void mlp_standardize(hipStream_t s, int n, const float *F, const float *mean, const float *sd, float *Z) {
    const int nb = (int)std::min<size_t>(1024, ((size_t)n * NIN + 255) / 256);
    hipLaunchKernelGGL(k_standardize, dim3(nb), dim3(256), 0, s, n, F, mean, sd, Z);
}
void mlp_gather(hipStream_t s, int cnt, const int *perm, const float *Z, const int *y, float *Zb, int *yb) {
    const int nb = std::min(1024, (cnt * NIN + 255) / 256);
    hipLaunchKernelGGL(k_gather_rows, dim3(nb), dim3(256), 0, s, cnt, perm, Z, y, Zb, yb);
}

}  // namespace sylv

using namespace sylv;

static float *g_mlp_scratch = nullptr;
static size_t g_mlp_scratch_n = 0;

extern "C" int sylv_mlp_forward(int n, const float *feats, const float *params, float *probs,
                                void *stream) {
    if (n < 0) return -1;
    if (n > 0 && !feats) return -2;
    if (!params) return -3;
    if (n > 0 && !probs) return -4;
    if (n == 0) return 0;
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_forward, dim3((n + 255) / 256), dim3(256), 0, s, n, feats, params, probs);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}

extern "C" int sylv_mlp_train_step(int n, const float *feats, const int *labels, float *params,
                                   float *adam_m, float *adam_v, int t, float lr, float *grad,
                                   float *loss, void *stream) {
    if (n <= 0) return -1;
    if (!feats) return -2;
    if (!labels) return -3;
    if (!params) return -4;
    if (!adam_m) return -5;
    if (!adam_v) return -6;
    if (t < 1) return -7;
    hipStream_t s = (hipStream_t)stream;
    const int nblk = (n + SPB - 1) / SPB;
    size_t need = (size_t)nblk * NPAR + n + 64;
    if (g_mlp_scratch_n < need) {
        if (g_mlp_scratch) hipFree(g_mlp_scratch);
        g_mlp_scratch = nullptr;
        g_mlp_scratch_n = 0;
        if (hipMalloc(&g_mlp_scratch, need * sizeof(float)) != hipSuccess) return SYLV_ERR_ALLOC;
        g_mlp_scratch_n = need;
    }
    float *part = g_mlp_scratch;
    float *lossv = part + (size_t)nblk * NPAR;
    float *lsum = lossv + n;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nblk), dim3(256), 0, s, n, feats, labels, params, part, lossv);
    hipLaunchKernelGGL(k_mlp_adam, dim3((NPAR + 255) / 256), dim3(256), 0, s, n, nblk, part, params,
                       adam_m, adam_v, t, lr, grad);
    if (loss) {
        hipLaunchKernelGGL(k_sum_loss, dim3(1), dim3(256), 0, s, n, lossv, lsum);
        hipError_t e = hipMemcpyAsync(loss, lsum, sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    }
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}
