// Learned precision selector: installed weights and the per-equation choice.
//
// The network (16-64-64-3, ReLU, softmax; forward and training kernels in
// mlp.hip) maps the 16 features of the low-precision Schur forms to a class:
// 0 = BF16-update forms + binary64 refinement, 1 = binary32 forms + binary64
// refinement, 2 = plain binary64.  The choice is advisory: the residual test
// of the refinement overrules it (escalation BF16 -> FP32 -> FP64).
#include "common.hpp"
#include "kernels.hpp"
#include "../../include/sylv.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <random>
#include <vector>

namespace sylv {

static std::mutex g_sel_mu;
static std::vector<float> g_sel;  // params, 16 feature means, 16 feature standard deviations
static int g_sel_version = 0;
struct SelDev {
    float *buf = nullptr;  // params | standardised features | probabilities
    int version = -1;
};
static SelDev g_seldev[64];

bool selector_installed() {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    return !g_sel.empty();
}

// Device buffer of the current device with the installed blob (params |
// means | deviations) up to date (uploaded on s when stale; caller holds no
// selector lock).
static float *selector_sync_device(hipStream_t s, int *rc) {
    *rc = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) { *rc = SYLV_ERR_NOGPU; return nullptr; }
    SelDev &d = g_seldev[dev];
    const size_t np = SYLV_MLP_NPARAM;
    if (!d.buf) {
        if (hipMalloc((void **)&d.buf, sizeof(float) * (np + 96)) != hipSuccess) { *rc = SYLV_ERR_ALLOC; return nullptr; }
        d.version = -1;
    }
    if (d.version != g_sel_version) {
        const hipError_t e = hipMemcpyAsync(d.buf, g_sel.data(), sizeof(float) * (np + 2 * SYLV_NFEAT),
                                            hipMemcpyHostToDevice, s);
        if (e == hipSuccess) {
            // the host blob can change after this call returns: finish the copy
            const hipError_t e2 = hipStreamSynchronize(s);
            if (e2 != hipSuccess) { *rc = SYLV_ERR_HIP - (int)e2; return nullptr; }
        } else {
            *rc = SYLV_ERR_HIP - (int)e;
            return nullptr;
        }
        d.version = g_sel_version;
    }
    return d.buf;
}

const float *selector_device_blob(hipStream_t s, int *rc) {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (g_sel.empty()) { *rc = -1; return nullptr; }
    return selector_sync_device(s, rc);
}

int selector_choose(hipStream_t s, char *hbuf, const float *f, int *cls, float *probs) {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (g_sel.empty()) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    SelDev &d = g_seldev[dev];
    const size_t np = SYLV_MLP_NPARAM;
    hipError_t e;
    int rc0 = 0;
    if (!selector_sync_device(s, &rc0)) return rc0;
    // device buffer: params | mean (16) | std (16) | raw features (16) |
    // standardised features (16) | probabilities (3)
    float *hb = reinterpret_cast<float *>(hbuf);
    float *dmean = d.buf + np, *dstd = dmean + SYLV_NFEAT, *draw = dstd + SYLV_NFEAT, *dz = draw + SYLV_NFEAT;
    float *dprob = dz + SYLV_NFEAT;
    for (int k = 0; k < SYLV_NFEAT; ++k) hb[k] = f[k];
    if ((e = hipMemcpyAsync(draw, hb, sizeof(float) * SYLV_NFEAT, hipMemcpyHostToDevice, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    mlp_standardize(s, 1, draw, dmean, dstd, dz);
    int rc = sylv_mlp_forward(1, dz, d.buf, dprob, s);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(hb + 32, dprob, sizeof(float) * SYLV_NCLASS, hipMemcpyDeviceToHost, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return SYLV_ERR_HIP - (int)e;
    int best = 0;
    for (int k = 0; k < SYLV_NCLASS; ++k) {
        probs[k] = hb[32 + k];
        if (hb[32 + k] > hb[32 + best]) best = k;
    }
    *cls = best;
    return 0;
}

}  // namespace sylv

using namespace sylv;

extern "C" int sylv_selector_set(const float *blob, int nvalues) {
    if (nvalues == 0) {  // uninstall
        std::lock_guard<std::mutex> lk(g_sel_mu);
        g_sel.clear();
        ++g_sel_version;
        return 0;
    }
    if (!blob) return -1;
    if (nvalues != SYLV_MLP_NPARAM + 2 * SYLV_NFEAT) return -2;
    for (int i = 0; i < nvalues; ++i)
        if (!std::isfinite(blob[i])) return -1;
    std::lock_guard<std::mutex> lk(g_sel_mu);
    g_sel.assign(blob, blob + nvalues);
    ++g_sel_version;
    return 0;
}

// Weights file (little-endian): 8 bytes "SYLVSEL1", int32 nparam (5443),
// int32 nfeat (16), int32 nclass (3), then nparam + 2 nfeat binary32 values
// (params, feature means, feature standard deviations).
extern "C" int sylv_selector_load(const char *path) {
    if (!path) return -1;
    FILE *fp = std::fopen(path, "rb");
    if (!fp) return -1;
    char magic[8];
    int32_t hdr[3];
    std::vector<float> blob(SYLV_MLP_NPARAM + 2 * SYLV_NFEAT);
    const bool ok = std::fread(magic, 1, 8, fp) == 8 && std::fread(hdr, sizeof(int32_t), 3, fp) == 3;
    int rc = 0;
    if (!ok || std::memcmp(magic, "SYLVSEL1", 8) != 0 || hdr[0] != SYLV_MLP_NPARAM || hdr[1] != SYLV_NFEAT ||
        hdr[2] != SYLV_NCLASS)
        rc = -2;
    else if (std::fread(blob.data(), sizeof(float), blob.size(), fp) != blob.size())
        rc = -2;
    std::fclose(fp);
    if (rc) return rc;
    rc = sylv_selector_set(blob.data(), (int)blob.size());
    return rc == -1 ? -3 : rc;
}

// Training on the GPU: per-feature mean and standard deviation of the raw
// features (k_feat_stats), standardisation (mlp_standardize), He-normal
// initialisation from a seeded host generator, then epochs of shuffled
// mini-batches (gathered on the device) through sylv_mlp_train_step.
extern "C" int sylv_selector_train(int n_samples, const float *feats, const int *labels,
                                   const sylv_train_opts *topts, float *weights_out, float *loss_hist,
                                   void *stream) {
    if (n_samples <= 0) return -1;
    if (!feats) return -2;
    if (!labels) return -3;
    sylv_train_opts o;
    sylv_default_train_opts(&o);
    if (topts) o = *topts;
    if (o.epochs < 0 || o.batch <= 0 || !(o.lr > 0.f)) return -4;
    if (!weights_out) return -5;
    hipStream_t s = (hipStream_t)stream;
    const int np = SYLV_MLP_NPARAM, nf = SYLV_NFEAT;
    const int bsz = std::min(o.batch, n_samples);
    float *work = nullptr;
    const size_t nwork = (size_t)n_samples * nf + (size_t)bsz * nf + 2 * (size_t)np + 64;
    int *iwork = nullptr;
    if (hipMalloc((void **)&work, nwork * sizeof(float)) != hipSuccess) return SYLV_ERR_ALLOC;
    if (hipMalloc((void **)&iwork, sizeof(int) * ((size_t)n_samples + bsz)) != hipSuccess) {
        hipFree(work);
        return SYLV_ERR_ALLOC;
    }
    float *Z = work, *Zb = Z + (size_t)n_samples * nf, *am = Zb + (size_t)bsz * nf, *av = am + np;
    int *perm = iwork, *yb = iwork + n_samples;
    float *params = weights_out, *mean = weights_out + np, *sd = mean + nf;
    int rc = 0;
    hipError_t e = hipSuccess;
    // He-normal initial weights (biases zero)
    std::vector<float> init(np, 0.f);
    std::mt19937_64 gen(o.seed);
    auto he = [&](int off, int rows, int cols) {
        std::normal_distribution<double> nd(0.0, std::sqrt(2.0 / cols));
        for (int k = 0; k < rows * cols; ++k) init[off + k] = (float)nd(gen);
    };
    he(0, 64, 16);
    he(64 * 16 + 64, 64, 64);
    he(64 * 16 + 64 + 64 * 64 + 64, 3, 64);
    std::vector<int> hperm(n_samples);
    for (int i = 0; i < n_samples; ++i) hperm[i] = i;
    do {
        mlp_feature_stats(s, n_samples, feats, mean, sd);
        mlp_standardize(s, n_samples, feats, mean, sd, Z);
        if ((e = hipMemcpyAsync(params, init.data(), sizeof(float) * np, hipMemcpyHostToDevice, s)) != hipSuccess)
            break;
        if ((e = hipMemsetAsync(am, 0, sizeof(float) * 2 * np, s)) != hipSuccess) break;
        int step = 0;
        for (int ep = 0; ep < o.epochs && !rc && e == hipSuccess; ++ep) {
            std::shuffle(hperm.begin(), hperm.end(), gen);
            // the host permutation must stay alive until the copy is done
            if ((e = hipMemcpyAsync(perm, hperm.data(), sizeof(int) * n_samples, hipMemcpyHostToDevice, s)) !=
                hipSuccess)
                break;
            double lsum = 0.0;
            int nb = 0;
            for (int b0 = 0; b0 < n_samples; b0 += bsz) {
                const int cnt = std::min(bsz, n_samples - b0);
                mlp_gather(s, cnt, perm + b0, Z, labels, Zb, yb);
                float loss = 0.f;
                rc = sylv_mlp_train_step(cnt, Zb, yb, params, am, av, ++step, o.lr, nullptr,
                                         loss_hist ? &loss : nullptr, s);
                if (rc) break;
                lsum += loss;
                ++nb;
            }
            if (loss_hist && nb) loss_hist[ep] = (float)(lsum / nb);
            if ((e = hipStreamSynchronize(s)) != hipSuccess) break;
        }
    } while (false);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    hipFree(work);
    hipFree(iwork);
    if (rc) return rc;
    if (e != hipSuccess) return SYLV_ERR_HIP - (int)e;
    e = hipGetLastError();
    return e == hipSuccess ? 0 : SYLV_ERR_HIP - (int)e;
}

extern "C" void sylv_default_train_opts(sylv_train_opts *o) {
    if (!o) return;
    o->epochs = 30;
    o->batch = 512;
    o->lr = 1e-3f;
    o->seed = 0;
}
