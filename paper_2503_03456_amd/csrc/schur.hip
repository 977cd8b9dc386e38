// Host driver of the real Schur factorisation A = U T U^T on one GPU:
// blocked Hessenberg reduction, then the small-bulge multishift QR algorithm
// with aggressive early deflation (Braman, Byers & Mathias 2002), using the
// single-workgroup LDS kernels of hqr.hip for the sequential parts and MFMA
// GEMMs for every update outside the current LDS window.
//
// Loop on the active block [ktop, kbot] (kbot starts at n-1):
//   - find the largest negligible subdiagonal entry above kbot -> ktop;
//   - blocks of order 1 and 2 are finished directly (2x2 with real
//     eigenvalues split by one rotation);
//   - blocks small enough for one workgroup are finished by one full-window
//     Schur kernel;
//   - otherwise: AED on a trailing window, then (unless AED deflated enough)
//     one multishift sweep with shifts taken from the undeflated window
//     eigenvalues (exceptional shifts after 6 sweeps without deflation).
// The host reads back a few integers and shifts per iteration.
#include "common.hpp"
#include "kernels.hpp"
#include "schur.hpp"

#include <array>
#include "prof.hpp"

#include <vector>
#include <cmath>
#include <cstdio>
#include <atomic>
#include <mutex>
#include <cstdlib>
#include <algorithm>

namespace sylv {

// current tunables (defaults measured on MI355X by the autotuner)
static std::mutex g_tune_mu;
static bool g_tune_set[2] = {false, false};
static SchurTune g_tune[2];
static SchurTune tune_default(bool fp32) {
    // selected by paper_2503_03456_amd.autotune (n = 2048, normal recipe,
    // seed 7) after the bulge chains were added: Schur time 0.250 -> 0.217 s
    // (binary32: 3 chains over 40 bulges, AED window 64), 0.368 -> 0.340 s
    // (binary64: 2 chains over 24 bulges)
    return fp32 ? SchurTune{64, 64, 40, 48, 50, 7, 8, 3} : SchurTune{64, 64, 24, 48, 40, 7, 16, 2};
}
template <typename T>
SchurTune schur_tune() {
    const int f = sizeof(T) == 4 ? 1 : 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune_set[f] ? g_tune[f] : tune_default(f == 1);
}
template <typename T>
int schur_tune_set(const SchurTune &t) {
    typedef SchurCaps<T> K;
    if (t.nsmall < 16 || t.nsmall > K::NSMALL) return -1;
    if (t.nw < 8 || t.nw > K::NSMALL) return -1;
    if (t.chains < 1 || t.chains > kChaseMaxWin) return -1;
    if (t.nb < 1 || t.nb > K::NBMAX) return -1;
    const int nbc = (t.nb + t.chains - 1) / t.chains;   // bulges of the largest chain
    if (t.adv < 4 || t.adv + 3 * nbc + 1 > K::WMAX) return -1;
    if (t.nibble < 0 || t.nibble > 100) return -1;
    if (t.aedw != 4 && t.aedw != 7) return -1;
    if (t.chasew != 8 && t.chasew != 16) return -1;
    if (aed_smem<T>(t.nw) > 160 * 1024) return -1;
    if (chase_smem<T>(t.adv + 3 * nbc + 1, nbc) > 160 * 1024) return -1;
    const int f = sizeof(T) == 4 ? 1 : 0;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[f] = t;
    g_tune_set[f] = true;
    return 0;
}
template SchurTune schur_tune<float>();
template SchurTune schur_tune<double>();
template int schur_tune_set<float>(const SchurTune &);
template int schur_tune_set<double>(const SchurTune &);

template <typename T>
size_t schur_work_bytes(int n) {
    typedef SchurCaps<T> K;
    const int wmax = K::WMAX;
    const int wide = std::max(wmax, K::NSMALL);
    size_t e = hessenberg_work_elems<T>(n, K::HNB, K::HS) + (size_t)K::NSMALL * K::NSMALL +
               (size_t)kChaseMaxWin * wmax * wmax + (size_t)wide * n + 3 * K::NBMAX + 64;
    return e * sizeof(T) + 1024;
}
template size_t schur_work_bytes<float>(int);
template size_t schur_work_bytes<double>(int);

namespace {

template <typename T>
struct Ctx {
    hipStream_t s;
    int n;
    T *H;
    int ldh;
    T *U;
    int ldu;
    T *hw, *Zw, *Uw, *tmp, *trd;
    char *hbuf;  // pinned host buffer (64 KiB): small kernel results, staged shifts
    int bf16;    // off-window updates with bfloat16 inputs (binary32 forms only)
};

template <typename T>
void carve(Ctx<T> &c, char *ws) {
    typedef SchurCaps<T> K;
    const int n = c.n;
    const int wmax = K::WMAX;
    const int wide = std::max(wmax, K::NSMALL);
    T *p = reinterpret_cast<T *>(ws);
    c.hw = p; p += hessenberg_work_elems<T>(n, K::HNB, K::HS);
    c.Zw = p; p += (size_t)K::NSMALL * K::NSMALL;
    c.Uw = p; p += (size_t)kChaseMaxWin * wmax * wmax;
    c.tmp = p; p += (size_t)wide * n;
    c.trd = p; p += 3 * K::NBMAX + 64;
}

// Layout of the pinned host buffer: the small-result kernels (k_find_ktop,
// k_aed, k_gather_sub) write their outputs there directly, so reading a
// result costs a stream synchronisation and no copy.
constexpr size_t HB_INT = 0;      // 8 ints: ktop / AED status and counters
constexpr size_t HB_WR = 512;     // AED shift candidates: wr, then wi (NSMALL each)
constexpr size_t HB_EXC = 4096;   // trailing diagonal / subdiagonal for exceptional shifts
constexpr size_t HB_TRD = 8192;   // shifts staged for upload

template <typename T>
hipError_t sync_host(Ctx<T> &c) {
    return hipStreamSynchronize(c.s);
}

// In-place window update on MFMA, all three regions in one launch:
//   H(w0:w0+w, w0+w:n) <- Z^T H(...)   strips of SS columns,
//   H(0:w0, w0:w0+w)   <- H(...) Z     strips of SS rows,
//   U(:, w0:w0+w)      <- U(...) Z     strips of SS rows.
// Each product reads only its own strip (w <= WMAX rows or columns), so a
// workgroup caches the whole strip in LDS, multiplies and writes it back in
// place: no temporary and no copy-back.  Z is staged whole in LDS too
// (dynamic shared memory: 121 KiB binary32, 131 KiB binary64, one workgroup
// per CU); the four wavefronts then take the 16x16 output blocks in turn
// with no further barrier.
// largest divisor of x that is <= cap
constexpr int div_le(int x, int cap) { return (x % cap == 0) ? cap : div_le(x, cap - 1); }

// LDS geometry for windows up to WPX wide (WPX a multiple of 16): the
// narrow form serves the chain, AED and small-block windows (<= 96),
// the wide one the rest (<= WMAX rounded up to 16).
template <typename T, int WPX>
struct WinLds {
    static constexpr int WP = WPX;
    static constexpr int SS = sizeof(T) == 4 ? 64 : 32;
    static constexpr int LDK = WP + 1, LDI = SS + 1, LDZ = WP + 1;
    static constexpr int SZ = (SS * LDK > WP * LDI) ? SS * LDK : WP * LDI;
    static constexpr size_t bytes = sizeof(T) * ((size_t)SZ + (size_t)WP * LDZ);
    // loads in flight per thread in the strip and Z staging (exact trip counts)
    static constexpr int UL = div_le(SS * WP / 256, 14), UZ = div_le(WP * WP / 256, 9);
};
template <typename T>
constexpr int win_wide() { return ((SchurCaps<T>::WMAX + 15) / 16) * 16; }
constexpr int kWinNarrow = 96;

// Window transforms of one launch: window g (rows/cols [w0[g], w0[g] + w[g]),
// factor Z[g]) has nl[g] left strips, nr[g] strips of H rows above it and
// nu[g] strips of U rows.  mode 0: every part of every window; mode 1: the
// left and U parts; mode 2: the right parts.  (Windows on disjoint rows and
// columns conflict only in H(window g', window g) for g' above g, which
// takes Z_g'^T from the left and Z_g from the right: mode 1 then mode 2.)
template <typename T>
struct WinSet {
    int w0[kChaseMaxWin], w[kChaseMaxWin], nl[kChaseMaxWin], nr[kChaseMaxWin], nu[kChaseMaxWin];
    const T *Z[kChaseMaxWin];
    int nwin, mode;
};

template <typename T, int WPX>
__global__ __launch_bounds__(256) void k_win_update(int n, T *H, int ldh, T *U, int ldu, WinSet<T> set) {
    typedef typename mfma16<T>::v4 v4;
    // this workgroup's window g and part: b < nl left, then right strips of
    // H, then strips of U (mode 1 skips the right strips, mode 2 has only them)
    int b = blockIdx.x, g = 0;
    for (;; ++g) {
        const int cnt = set.mode == 0 ? set.nl[g] + set.nr[g] + set.nu[g]
                        : set.mode == 1 ? set.nl[g] + set.nu[g] : set.nr[g];
        if (b < cnt || g == set.nwin - 1) break;
        b -= cnt;
    }
    const int w0 = set.w0[g], w = set.w[g];
    const T *__restrict__ Z = set.Z[g];
    int nl = set.nl[g], nr = set.nr[g];
    if (set.mode == 1) nr = 0;                   // b >= nl: U strips
    else if (set.mode == 2) b += nl;             // past the left range: right strip b - nl
    typedef WinLds<T, WPX> L;
    constexpr int WP = L::WP, SS = L::SS, LDK = L::LDK, LDI = L::LDI, LDZ = L::LDZ;
    constexpr int RB = SS / 16;   // 16x16 output blocks across the strip
    extern __shared__ __align__(16) unsigned char win_smem[];
    T *S = reinterpret_cast<T *>(win_smem);
    T *Zs = S + L::SZ;
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63;
    // k steps of 4, rounded up to whole groups of 4 steps: S and Zs are zero
    // from k = w up to WP, a multiple of 16
    const int nkk = (((w + 3) / 4) + 3) & ~3;
    const int nch = (w + 15) / 16;
    // Staging: every thread issues UL (UZ) loads before their LDS stores, at
    // addresses clamped into the matrix, with exact trip counts and no
    // value-dependent selects, so nothing turns them back into one branch
    // and one wait per load.  Only Zs needs zeros outside w (rows k >= w, by
    // a 0/1 factor; Z is finite): with those, the strip's padding reaches
    // only outputs that are not stored.
    constexpr int UL = L::UL, UZ = L::UZ;
    static_assert((SS * WP) % (256 * UL) == 0 && (WP * WP) % (256 * UZ) == 0, "staging trip counts");
    const bool left = b < nl;
    T *M;
    int ldm, r0, c0, ext;   // strip origin in M and its extent (columns for left, rows for right)
    if (left) {
        M = H; ldm = ldh;
        r0 = w0;
        c0 = w0 + w + SS * b;
        ext = min(SS, n - c0);
        // S[j * LDK + k] = H(w0 + k, c0 + j)
        for (int e0 = tid; e0 < SS * WP; e0 += 256 * UL) {
            T v[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int e = e0 + 256 * u, k = e % WP, j = e / WP;
                v[u] = CM(M, r0 + (k < w ? k : w - 1), c0 + (j < ext ? j : ext - 1), ldm);
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int e = e0 + 256 * u;
                S[(e / WP) * LDK + e % WP] = v[u];
            }
        }
    } else {
        b -= nl;
        int rows;
        if (set.mode == 2 || b < nr) { M = H; ldm = ldh; rows = w0; }
        else { b -= nr; M = U; ldm = ldu; rows = n; }
        r0 = SS * b;
        c0 = w0;
        ext = min(SS, rows - r0);
        // S[k * LDI + i] = M(r0 + i, w0 + k)
        for (int e0 = tid; e0 < SS * WP; e0 += 256 * UL) {
            T v[UL];
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int e = e0 + 256 * u, i = e % SS, k = e / SS;
                v[u] = CM(M, r0 + (i < ext ? i : ext - 1), c0 + (k < w ? k : w - 1), ldm);
            }
#pragma unroll
            for (int u = 0; u < UL; ++u) {
                const int e = e0 + 256 * u;
                S[(e / SS) * LDI + e % SS] = v[u];
            }
        }
    }
    // Zs[j * LDZ + k] = Z(k, j) for k < w, zero for k >= w (all WP columns j)
    for (int e0 = tid; e0 < WP * WP; e0 += 256 * UZ) {
        T v[UZ];
#pragma unroll
        for (int u = 0; u < UZ; ++u) {
            const int e = e0 + 256 * u, k = e % WP, j = e / WP;
            v[u] = Z[(size_t)(j < w ? j : w - 1) * w + (k < w ? k : w - 1)] * T(k < w ? 1 : 0);
        }
#pragma unroll
        for (int u = 0; u < UZ; ++u) {
            const int e = e0 + 256 * u;
            Zs[(e / WP) * LDZ + e % WP] = v[u];
        }
    }
    __syncthreads();
    for (int blk = wv; blk < RB * nch; blk += 4) {
        const int ob = blk % RB, ch = blk / RB;
        const int bo = 16 * ob;   // first strip row (right) / column (left) of the block
        const T *zc = Zs + (16 * ch + (l & 15)) * LDZ;
        v4 acc = v4{0, 0, 0, 0};
        if (left) {
            // out(i, j) = sum_k Z(k, i) S(k, j): i in chunk ch, j in block ob
            const T *sp = S + (bo + (l & 15)) * LDK;
            for (int kk0 = 0; kk0 < nkk; kk0 += 4) {
                T sa[4], za[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * (kk0 + u) + (l >> 4);
                    sa[u] = sp[k]; za[u] = zc[k];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) acc = mfma16<T>::op(sa[u], za[u], acc);
            }
            const int i = 16 * ch + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = bo + mfma16<T>::orow(l, r);
                if (i < w && j < ext) CM(M, r0 + i, c0 + j, ldm) = acc[r];
            }
        } else {
            // out(i, j) = sum_k S(i, k) Z(k, j): i in block ob, j in chunk ch
            const T *sp = S + bo + (l & 15);
            for (int kk0 = 0; kk0 < nkk; kk0 += 4) {
                T sa[4], za[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int k = 4 * (kk0 + u) + (l >> 4);
                    sa[u] = sp[k * LDI]; za[u] = zc[k];
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) acc = mfma16<T>::op(za[u], sa[u], acc);
            }
            const int i = bo + (l & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 16 * ch + mfma16<T>::orow(l, r);
                if (i < ext && j < w) CM(M, r0 + i, c0 + j, ldm) = acc[r];
            }
        }
    }
}

// raises k_win_update's dynamic-LDS limits once per element type
template <typename T>
bool win_lds_ready() {
    static std::once_flag once;
    static bool ok = false;
    std::call_once(once, [] {
        ok = hipFuncSetAttribute((const void *)k_win_update<T, win_wide<T>()>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)WinLds<T, win_wide<T>()>::bytes) == hipSuccess &&
             hipFuncSetAttribute((const void *)k_win_update<T, kWinNarrow>,
                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)WinLds<T, kWinNarrow>::bytes) == hipSuccess;
        if (!ok) (void)hipGetLastError();
    });
    return ok;
}

// one launch of k_win_update over set: the narrow LDS form when every
// window of the set fits it
template <typename T>
void win_launch(Ctx<T> &c, const WinSet<T> &set, int grid) {
    if (grid <= 0) return;
    int wmax = 0;
    for (int g = 0; g < set.nwin; ++g) wmax = std::max(wmax, set.w[g]);
    constexpr size_t nb = WinLds<T, kWinNarrow>::bytes, wb = WinLds<T, win_wide<T>()>::bytes;
    if (wmax <= kWinNarrow)
        hipLaunchKernelGGL((k_win_update<T, kWinNarrow>), dim3(grid), dim3(256), nb, c.s, c.n, c.H, c.ldh, c.U,
                           c.ldu, set);
    else
        hipLaunchKernelGGL((k_win_update<T, win_wide<T>()>), dim3(grid), dim3(256), wb, c.s, c.n, c.H, c.ldh, c.U,
                           c.ldu, set);
}

// strip counts of window slot g of a launch
template <typename T>
void win_counts(const Ctx<T> &c, WinSet<T> &set, int g, int w0, int w, const T *Z) {
    constexpr int SS = WinLds<T, kWinNarrow>::SS;
    const int nc = c.n - (w0 + w);
    set.w0[g] = w0;
    set.w[g] = w;
    set.Z[g] = Z;
    set.nl[g] = nc > 0 ? (nc + SS - 1) / SS : 0;
    set.nr[g] = (w0 + SS - 1) / SS;
    set.nu[g] = (c.n + SS - 1) / SS;
}

template <typename T>
void apply_window(Ctx<T> &c, int w0, int w, const T *Z);

// The transforms of several disjoint chain windows: left and U parts of
// all windows in one launch, then the right parts in a second.
template <typename T>
void apply_windows(Ctx<T> &c, const ChaseSet<T> &cs, int nwin) {
    bool fused = !c.bf16 && nwin > 1 && win_lds_ready<T>();
    for (int g = 0; g < nwin && fused; ++g) fused = cs.w[g].W <= SchurCaps<T>::WMAX;
    if (!fused) {
        for (int g = 0; g < nwin; ++g) apply_window(c, cs.w[g].ws, cs.w[g].W, cs.w[g].Uw);
        return;
    }
    WinSet<T> set;
    int nlu = 0, nr = 0;
    for (int g = 0; g < nwin; ++g) {
        win_counts(c, set, g, cs.w[g].ws, cs.w[g].W, cs.w[g].Uw);
        nlu += set.nl[g] + set.nu[g];
        nr += set.nr[g];
    }
    set.nwin = nwin;
    ProfScope ps(KID_WIN, c.s);
    set.mode = 1;
    win_launch(c, set, nlu);
    set.mode = 2;
    win_launch(c, set, nr);
}

// Apply a window transform Z (w x w, ld w) acting on rows/cols [w0, w0+w):
// H(w0:w0+w, w0+w:n) <- Z^T H(...), H(0:w0, w0:w0+w) <- H(...) Z,
// U(:, w0:w0+w) <- U(...) Z.  Binary32/binary64: the fused in-place kernel;
// the BF16 option keeps bfloat16-input GEMMs through a temporary.
template <typename T>
void apply_window(Ctx<T> &c, int w0, int w, const T *Z) {
    const int n = c.n;
    const int nc = n - (w0 + w);
    if (!c.bf16 && w <= SchurCaps<T>::WMAX && win_lds_ready<T>()) {
        WinSet<T> set;
        win_counts(c, set, 0, w0, w, Z);
        set.nwin = 1;
        set.mode = 0;
        ProfScope ps(KID_WIN, c.s);
        win_launch(c, set, set.nl[0] + set.nr[0] + set.nu[0]);
        return;
    }
    if (nc > 0) {
        T *blk = c.H + (size_t)(w0 + w) * c.ldh + w0;
        gemm<T, T, T, T>(c.s, 1, 0, w, nc, w, T(1), Z, w, blk, c.ldh, T(0), c.tmp, w, T(1), c.bf16);
        cast<T, T>(c.s, w, nc, c.tmp, w, blk, c.ldh, T(1));
    }
    if (w0 > 0) {
        T *blk = c.H + (size_t)w0 * c.ldh;
        gemm<T, T, T, T>(c.s, 0, 0, w0, w, w, T(1), blk, c.ldh, Z, w, T(0), c.tmp, w0, T(1), c.bf16);
        cast<T, T>(c.s, w0, w, c.tmp, w0, blk, c.ldh, T(1));
    }
    T *ub = c.U + (size_t)w0 * c.ldu;
    gemm<T, T, T, T>(c.s, 0, 0, n, w, w, T(1), ub, c.ldu, Z, w, T(0), c.tmp, n, T(1), c.bf16);
    cast<T, T>(c.s, n, w, c.tmp, n, ub, c.ldu, T(1));
}

// Pair shifts (wr[i] + i wi[i]) into bulges, three entries per bulge: a
// complex pair -> (re, |im|, 1); two reals -> (s1, s2, 0).
template <typename T>
void pair_shifts(const std::vector<double> &wr, const std::vector<double> &wi, int maxb,
                 std::vector<T> &trd) {
    trd.clear();
    std::vector<double> reals;
    // walk from the bottom (last entries are closest to kbot)
    int i = (int)wr.size() - 1;
    std::vector<std::array<double, 3>> bul;
    while (i >= 0 && (int)bul.size() < maxb) {
        if (wi[i] != 0.0 && i >= 1 && wi[i - 1] != 0.0) {
            bul.push_back({wr[i], std::fabs(wi[i]), 1.0});
            i -= 2;
        } else if (wi[i] != 0.0) {
            i -= 1;  // orphan half of a pair (cut window): skip
        } else {
            reals.push_back(wr[i]);
            if (reals.size() == 2) {
                bul.push_back({reals[0], reals[1], 0.0});
                reals.clear();
            }
            i -= 1;
        }
    }
    // the bulge introduced first should carry the shifts closest to the bottom
    for (auto &b : bul)
        for (int k = 0; k < 3; ++k) trd.push_back((T)b[k]);
}

}  // namespace

template <typename T>
int schur_run(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, char *ws, char *hbuf,
              int *qr_status, int bf16) {
    typedef SchurCaps<T> K;
    const SchurTune P = schur_tune<T>();
    *qr_status = 0;
    if (n <= 0) return 0;
    Ctx<T> c{s, n, H, ldh, U, ldu};
    c.hbuf = hbuf;
    c.bf16 = (sizeof(T) == sizeof(float)) ? bf16 : 0;
    carve(c, ws);
    hessenberg<T>(s, n, H, ldh, U, ldu, c.hw, K::HNB, K::HS, c.bf16);
    int *hi = reinterpret_cast<int *>(c.hbuf + HB_INT);
    T *hwr = reinterpret_cast<T *>(c.hbuf + HB_WR);
    T *hwi = hwr + K::NSMALL;
    static_assert(HB_WR + 2 * sizeof(T) * K::NSMALL <= HB_EXC && HB_EXC + sizeof(T) * (4 * K::NBMAX + 8) <= HB_TRD &&
                      schur_hbuf_bytes<T>() <= 65536,
                  "host buffer layout");
    hipError_t err;
    int kbot = n - 1;
    int ndfl = 1;
    long iters = 0;
    const long itmax = 100L + n / 2;  // AED + sweep rounds before giving up
    std::vector<double> wr, wi;
    std::vector<T> trd;
    // SYLV_TRACE=1: per-factorisation counters of the QR phase on stderr
    const bool trace = std::getenv("SYLV_TRACE") != nullptr;
    long st_aed = 0, st_sweeps = 0, st_chase = 0, st_fsw = 0, st_fst = 0, st_kcyc = 0, st_defl = 0;
    while (kbot >= 0) {
        find_ktop<T>(s, H, ldh, 0, kbot, hi);
        if ((err = sync_host(c)) != hipSuccess) return SYLV_ERR_HIP - (int)err;
        const int ktop = hi[0];
        const int N = kbot - ktop + 1;
        if (N == 1) { kbot -= 1; ndfl = 1; continue; }
        if (N == 2) { std2x2<T>(s, n, H, ldh, U, ldu, ktop); kbot -= 2; ndfl = 1; continue; }
        if (++iters > itmax) { *qr_status = 1; break; }
        if (N <= P.nsmall) {
            if (aed_launch<T>(s, N, H, ldh, ktop, 0, c.Zw, hi, hwr, hwi, P.aedw)) return -1;
            if ((err = sync_host(c)) != hipSuccess) return SYLV_ERR_HIP - (int)err;
            ++st_aed; st_fsw += hi[3]; st_fst += hi[4]; st_kcyc += hi[5];
            prof_add_work(KID_AED, 12.0 * (2.0 * N + 3.0) * hi[4]);
            if (hi[0] != 0) { *qr_status = 1; break; }
            apply_window(c, ktop, N, c.Zw);
            kbot = ktop - 1;
            ndfl = 1;
            continue;
        }
        // aggressive early deflation on the trailing window
        const int nw = std::min(P.nw, N - 1);
        const int kwtop = kbot - nw + 1;
        if (aed_launch<T>(s, nw, H, ldh, kwtop, 1, c.Zw, hi, hwr, hwi, P.aedw)) return -1;
        if ((err = sync_host(c)) != hipSuccess) return SYLV_ERR_HIP - (int)err;
        const int aed_st = hi[0], nd = hi[1], nsu = hi[2];
        ++st_aed; st_fsw += hi[3]; st_fst += hi[4]; st_kcyc += hi[5]; st_defl += nd;
        prof_add_work(KID_AED, 12.0 * (2.0 * nw + 3.0) * hi[4]);
        if (aed_st == 0) apply_window(c, kwtop, nw, c.Zw);
        // shift candidates: eigenvalues of the undeflated part of the window
        wr.clear(); wi.clear();
        if (aed_st == 0 && nsu > 0)
            for (int i = 0; i < nsu; ++i) { wr.push_back(hwr[i]); wi.push_back(hwi[i]); }
        const int ndef = (aed_st == 0) ? nd : 0;
        kbot -= ndef;
        ndfl = (ndef > 0) ? 1 : ndfl + 1;
        // skip the sweep if AED deflated a good share of the window
        if (ndef > 0 && 100 * ndef > P.nibble * nw) continue;
        if (kbot - ktop + 1 <= P.nsmall) continue;
        const int N2 = kbot - ktop + 1;
        const int maxb = std::min(P.nb, (N2 - 2) / 6 > 1 ? (N2 - 2) / 6 : 1);
        if (ndfl % 6 == 0 || wr.size() < 2) {
            // exceptional shifts from the trailing subdiagonal magnitudes
            const int cnt = 2 * maxb + 2;
            // H(i,i) and H(i,i-1) for i in [i0, kbot], and H(i0-1, i0-2)
            int i0 = std::max(ktop + 2, kbot - cnt + 1);
            int m = kbot - i0 + 1;
            T *hv = reinterpret_cast<T *>(c.hbuf + HB_EXC);
            gather_sub<T>(s, H, ldh, i0, m, hv);
            if ((err = sync_host(c)) != hipSuccess) return SYLV_ERR_HIP - (int)err;
            trd.clear();
            // exceptional pair aa +- i sqrt(0.4375) ss (the eigenvalues of
            // [[aa, -0.4375 ss], [ss, aa]])
            for (int q = m - 1; q >= 1 && (int)trd.size() < 3 * maxb; q -= 2) {
                double sub_i = std::fabs((double)hv[2 * q + 1]);
                double sub_im1 = std::fabs((double)hv[2 * (q - 1) + 1]);
                double ss = sub_i + sub_im1;
                double aa = 0.75 * ss + (double)hv[2 * q];
                trd.push_back((T)aa);
                trd.push_back((T)(std::sqrt(0.4375) * ss));
                trd.push_back(T(1));
            }
            if (trd.empty()) {
                double ss = std::fabs((double)hv[2 * m]);
                double aa = 0.75 * ss + (double)hv[2 * (m - 1)];
                trd.push_back((T)aa);
                trd.push_back((T)(std::sqrt(0.4375) * ss));
                trd.push_back(T(1));
            }
        } else {
            pair_shifts<T>(wr, wi, maxb, trd);
        }
        const int nb = (int)trd.size() / 3;
        if (nb == 0) continue;
        T *htrd = reinterpret_cast<T *>(c.hbuf + HB_TRD);
        for (size_t q = 0; q < trd.size(); ++q) htrd[q] = trd[q];
        hipMemcpyAsync(c.trd, htrd, sizeof(T) * trd.size(), hipMemcpyHostToDevice, s);
        // multishift sweep over [ktop, kbot]: the nb bulges form G chains
        // (the first chain, introduced first, carries the first shifts);
        // chain g enters D[g] steps after the sweep starts, one window width
        // of the chain below it later, so the chains' windows never overlap
        const int G = std::max(1, std::min(P.chains, nb));
        int cnb[kChaseMaxWin], cfb[kChaseMaxWin], D[kChaseMaxWin];
        for (int g = 0, f = 0; g < G; ++g) {
            cnb[g] = nb / G + (g < nb % G ? 1 : 0);
            cfb[g] = f;
            f += cnb[g];
            D[g] = g == 0 ? 0 : D[g - 1] + P.adv + 3 * cnb[g - 1] + 1;
        }
        const int ttot = D[G - 1] + (N2 - 2) + 3 * (cnb[G - 1] - 1) + 1;
        ++st_sweeps;
        const size_t wsq = (size_t)K::WMAX * K::WMAX;
        for (int t0 = 0; t0 < ttot; t0 += P.adv) {
            const int t1 = std::min(t0 + P.adv, ttot);
            ChaseSet<T> set;
            int nwin = 0;
            for (int g = 0; g < G; ++g) {
                const int r0 = t0 - D[g], r1 = t1 - D[g];   // chain time
                const int pmin = std::max(0, r0 - 3 * (cnb[g] - 1));
                const int pmax = std::min(N2 - 2, r1 - 1);
                if (pmax < pmin) continue;
                const int ws_ = ktop + std::max(0, pmin - 1);
                const int we_ = ktop + std::min(N2, pmax + 4);
                set.w[nwin] = ChaseWin<T>{ws_, we_ - ws_, r0, cnb[g], c.trd + 3 * cfb[g], c.Uw + nwin * wsq};
                ++nwin;
            }
            if (nwin == 0) continue;
            if (chase_launch<T>(s, H, ldh, ktop, kbot, set, nwin, t1 - t0, P.chasew)) return -1;
            ++st_chase;
            // the windows' updates commute (disjoint rows and columns except
            // H(window g', window g) for a window g' above g, which takes
            // Z_g'^T from the left and Z_g from the right): one after another
            apply_windows(c, set, nwin);
        }
        // no synchronisation here: the staged shifts are next rewritten after
        // the next find_ktop synchronisation, which follows their upload
    }
    clean_lower<T>(s, n, H, ldh);
    if (trace)
        std::fprintf(stderr,
                     "[sylv] schur<%s> n=%d: AED calls %ld (deflated %ld), sweeps %ld, chase "
                     "phases %ld, window Francis sweeps %ld steps %ld kcycles %ld (%.0f cycles/step)\n",
                     sizeof(T) == 4 ? "fp32" : "fp64", n, st_aed, st_defl, st_sweeps, st_chase, st_fsw,
                     st_fst, st_kcyc, st_fst ? 1024.0 * st_kcyc / st_fst : 0.0);
    return 0;
}
template int schur_run<float>(hipStream_t, int, float *, int, float *, int, char *, char *, int *, int);
template int schur_run<double>(hipStream_t, int, double *, int, double *, int, char *, char *, int *, int);

}  // namespace sylv
