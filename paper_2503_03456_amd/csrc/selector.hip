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
#include <mutex>
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

int selector_choose(hipStream_t s, char *hbuf, const float *f, int *cls, float *probs) {
    std::lock_guard<std::mutex> lk(g_sel_mu);
    if (g_sel.empty()) return -1;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return SYLV_ERR_NOGPU;
    SelDev &d = g_seldev[dev];
    const size_t np = SYLV_MLP_NPARAM;
    hipError_t e;
    if (!d.buf) {
        if (hipMalloc((void **)&d.buf, sizeof(float) * (np + 64)) != hipSuccess) return SYLV_ERR_ALLOC;
        d.version = -1;
    }
    float *hb = reinterpret_cast<float *>(hbuf);
    if (d.version != g_sel_version) {
        if ((e = hipMemcpyAsync(d.buf, g_sel.data(), sizeof(float) * np, hipMemcpyHostToDevice, s)) != hipSuccess)
            return SYLV_ERR_HIP - (int)e;
        d.version = g_sel_version;
    }
    const float *mean = g_sel.data() + np, *sd = mean + SYLV_NFEAT;
    for (int k = 0; k < SYLV_NFEAT; ++k) hb[k] = (f[k] - mean[k]) / (sd[k] > 0.f ? sd[k] : 1.f);
    if ((e = hipMemcpyAsync(d.buf + np, hb, sizeof(float) * SYLV_NFEAT, hipMemcpyHostToDevice, s)) != hipSuccess)
        return SYLV_ERR_HIP - (int)e;
    int rc = sylv_mlp_forward(1, d.buf + np, d.buf, d.buf + np + 32, s);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(hb + 32, d.buf + np + 32, sizeof(float) * SYLV_NCLASS, hipMemcpyDeviceToHost, s)) !=
        hipSuccess)
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
