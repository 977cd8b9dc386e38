// MFMA GEMM for gfx950: C = alpha * op(A) * op(B) + beta * C, column-major.
//
// One kernel template serves every precision pair the solver needs:
//   ACC = double -> v_mfma_f64_16x16x4f64 (binary64 residual, plain FP64 path)
//   ACC = float  -> v_mfma_f32_16x16x4f32 (binary32 Schur updates, transforms)
// Operands may be stored in a wider type than ACC (binary64 residual read
// straight into a binary32 product: the conversion happens on the way into
// LDS) and C may be wider than ACC (binary64 X += binary32 product).
//
// Tiling: 64x64 output tile per 256-thread workgroup (4 wave64s in a 2x2
// grid, each 32x32 = 2x2 MFMA blocks of 16x16), K staged through LDS 16 at a
// time with a register prefetch of the next K slice.  The MFMA operands are
// fed swapped (op(B)^T in the A slot, op(A)^T in the B slot) so that each
// lane's accumulators run down a column of C: stores are 16 consecutive
// elements of a column per quarter-wave.
#include <cstdlib>
#include <type_traits>
#include "common.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace sylv {

constexpr int GBM = 64, GBN = 64, GBK = 16, GPAD = 16;

// One 64x64 output tile (rows row0.., cols col0..) of C = alpha op(A) op(B) + beta C.
template <typename TA, typename TB, typename TC, typename ACC>
SYLV_DEVINL void gemm_tile(int M, int N, int K, const TA *__restrict__ A, int lda, int ta,
                           const TB *__restrict__ B, int ldb, int tb, TC *__restrict__ C, int ldc,
                           double alpha, ACC beta, TB bscale, int row0, int col0,
                           ACC (&As)[GBK][GBM + GPAD], ACC (&Bs)[GBK][GBN + GPAD]) {
    typedef typename mfma16<ACC>::v4 v4;

    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;

    v4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = v4{0, 0, 0, 0};

    // the next slab is held in registers in its storage format and scaled
    // and converted only when written to LDS: nothing waits on the loads
    // until the MFMAs of the current slab have been issued
    TA ra[4];
    TB rb[4];
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i, k;
            if (!ta) { i = l; k = (t >> 6) + 4 * r; } else { k = t & 15; i = (t >> 4) + 16 * r; }
            int gi = row0 + i, gk = k0 + k;
            TA v = TA(0);
            if (gi < M && gk < K) v = ta ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi];
            ra[r] = v;
            int j;
            if (!tb) { k = t & 15; j = (t >> 4) + 16 * r; } else { j = l; k = (t >> 6) + 4 * r; }
            int gj = col0 + j;
            gk = k0 + k;
            TB u = TB(0);
            if (gj < N && gk < K) u = tb ? B[(size_t)gk * ldb + gj] : B[(size_t)gj * ldb + gk];
            rb[r] = u;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int i, k;
            if (!ta) { i = l; k = (t >> 6) + 4 * r; } else { k = t & 15; i = (t >> 4) + 16 * r; }
            As[k][i] = (ACC)ra[r];
            int j;
            if (!tb) { k = t & 15; j = (t >> 4) + 16 * r; } else { j = l; k = (t >> 6) + 4 * r; }
            // the scale (a power of two) is applied in the storage precision
            // before the conversion, which keeps the range
            Bs[k][j] = (ACC)(bscale * rb[r]);
        }
    };

    const int nk = (K + GBK - 1) / GBK;
    if (nk > 0) load(0);
    for (int kt = 0; kt < nk; ++kt) {
        store();
        __syncthreads();
        if (kt + 1 < nk) load((kt + 1) * GBK);
#pragma unroll
        for (int kk = 0; kk < GBK / 4; ++kk) {
            const int kr = 4 * kk + (l >> 4);
            ACC fa[2], fb[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) fa[a] = As[kr][32 * wm + 16 * a + (l & 15)];
#pragma unroll
            for (int b = 0; b < 2; ++b) fb[b] = Bs[kr][32 * wn + 16 * b + (l & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma16<ACC>::op(fb[b], fa[a], acc[a][b]);
        }
        __syncthreads();
    }

#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int i = row0 + 32 * wm + 16 * a + (l & 15);
                int j = col0 + 32 * wn + 16 * b + mfma16<ACC>::orow(l, r);
                if (i < M && j < N) {
                    // alpha is applied in the precision of C: a binary64 C
                    // takes an un-scaling power of two without binary32
                    // overflow or underflow
                    TC *p = C + (size_t)j * ldc + i;
                    const TC v = (TC)alpha * (TC)acc[a][b][r];
                    if (beta != ACC(0)) *p = v + (TC)beta * (*p);
                    else *p = v;
                }
            }
}

// ------------------------------------------------------ 128 x 128 tiles
// Large products (M, N >= 1024-ish, K >= 256): a 128 x 128 output tile per 256-thread
// workgroup, each wave64 a 64 x 64 quadrant (4 x 4 MFMA blocks of 16 x 16),
// K staged through two LDS buffers 32 at a time (one barrier per K step: a
// buffer is rewritten only after every wave has passed the barrier that
// follows its last read).  Global loads move 8 consecutive elements per
// thread along the contiguous dimension of each operand, as 16-byte vector
// loads when the operand's base and leading dimension allow it.
constexpr int LBM = 128, LBK = 32, LPAD = 16, LLD = LBM + LPAD;

// 8 consecutive elements p[0..7] (cnt of them in range, zeros after) in
// their storage format; the caller scales and converts them when it writes
// the slab to LDS, so the loads stay in flight across the current slab's
// MFMAs
template <typename TS>
SYLV_DEVINL void load8(const TS *p, int cnt, bool vec, TS (&out)[8]) {
    if (vec && cnt >= 8) {
        if constexpr (sizeof(TS) == 8) {
            typedef double d2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const d2 v = *reinterpret_cast<const d2 *>(p + 2 * h);
                out[2 * h] = v[0];
                out[2 * h + 1] = v[1];
            }
        } else {
            typedef float f4 __attribute__((ext_vector_type(4)));
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const f4 v = *reinterpret_cast<const f4 *>(p + 4 * h);
#pragma unroll
                for (int z = 0; z < 4; ++z) out[4 * h + z] = v[z];
            }
        }
        return;
    }
#pragma unroll
    for (int h = 0; h < 8; ++h) out[h] = (h < cnt) ? p[h] : TS(0);
}

template <typename TA, typename TB, typename TC, typename ACC, int ta, int tb>
__global__ __launch_bounds__(256) void gemm128_kernel(int M, int N, int K, const TA *__restrict__ A, int lda,
                                                      const TB *__restrict__ B, int ldb, TC *__restrict__ C,
                                                      int ldc, double alpha, ACC beta, int tiles_m, TB bscale,
                                                      int upper) {
    typedef typename mfma16<ACC>::v4 v4;
    __shared__ ACC As[2][LBK][LLD];
    __shared__ ACC Bs[2][LBK][LLD];
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    // workgroups are dealt to the 8 XCDs round-robin: renumber so that each
    // XCD takes a consecutive run of nblk / 8 tiles
    if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    int tm, tn;
    if (upper) sym_pair_index(bid, tm, tn);
    else {
        // tiles in groups of G tile rows, column by column inside a group:
        // each XCD's run of tiles is then a block about G rows tall rather
        // than whole tile columns, so its L2 sees fewer distinct rows of
        // op(A) for the same columns of op(B)
        constexpr int G = 4;
        const int tiles_n = nblk / tiles_m, per = G * tiles_n;
        const int grp = bid / per, m0 = grp * G, gs = min(G, tiles_m - m0), r = bid - grp * per;
        tm = m0 + r % gs;
        tn = r / gs;
    }
    const int row0 = tm * LBM, col0 = tn * LBM;
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;
    // vector loads need 16-byte aligned columns
    const bool va = ((reinterpret_cast<size_t>(A) | ((size_t)lda * sizeof(TA))) & 15) == 0;
    const bool vb = ((reinterpret_cast<size_t>(B) | ((size_t)ldb * sizeof(TB))) & 15) == 0;
    // coordinates of this thread's 8 consecutive elements in each 16-deep
    // half of the slab
    //   op(A) 128 x 16: !ta -> rows ai..ai+7 of column ak; ta -> k ak..ak+7 of row ai
    //   op(B) 16 x 128: !tb -> k bk..bk+7 of column bj; tb -> columns bj..bj+7 of row bk
    const int ai = ta ? (t >> 1) : (t & 15) * 8, ak = ta ? (t & 1) * 8 : (t >> 4);
    const int bj = tb ? (t & 15) * 8 : (t >> 1), bk = tb ? (t >> 4) : (t & 1) * 8;
    constexpr int KH = LBK / 16;   // 16-deep halves of the slab per thread
    TA ra[KH][8];
    TB rb[KH][8];
    auto load = [&](int k0) {
#pragma unroll
        for (int hh = 0; hh < KH; ++hh) {
            const int kb = k0 + 16 * hh;
            if constexpr (!ta) {
                const int gi = row0 + ai, gk = kb + ak;
                const int cnt = (gk < K) ? min(8, M - gi) : 0;
                load8<TA>(A + (size_t)gk * lda + gi, cnt > 0 ? cnt : 0, va, ra[hh]);
            } else {
                const int gi = row0 + ai, gk = kb + ak;
                const int cnt = (gi < M) ? min(8, K - gk) : 0;
                load8<TA>(A + (size_t)gi * lda + gk, cnt > 0 ? cnt : 0, va, ra[hh]);
            }
            if constexpr (!tb) {
                const int gj = col0 + bj, gk = kb + bk;
                const int cnt = (gj < N) ? min(8, K - gk) : 0;
                load8<TB>(B + (size_t)gj * ldb + gk, cnt > 0 ? cnt : 0, vb, rb[hh]);
            } else {
                const int gj = col0 + bj, gk = kb + bk;
                const int cnt = (gk < K) ? min(8, N - gj) : 0;
                load8<TB>(B + (size_t)gk * ldb + gj, cnt > 0 ? cnt : 0, vb, rb[hh]);
            }
        }
    };
    auto store = [&](int st) {
#pragma unroll
        for (int hh = 0; hh < KH; ++hh)
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                // B's scale (a power of two) in its storage precision, then
                // the conversion
                const ACC av = (ACC)ra[hh][h], bv = (ACC)(bscale * rb[hh][h]);
                if constexpr (!ta) As[st][16 * hh + ak][ai + h] = av;
                else As[st][16 * hh + ak + h][ai] = av;
                if constexpr (!tb) Bs[st][16 * hh + bk + h][bj] = bv;
                else Bs[st][16 * hh + bk][bj + h] = bv;
            }
    };
    v4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = v4{0, 0, 0, 0};
    const int nk = (K + LBK - 1) / LBK;
    if (nk > 0) load(0);
    for (int kt = 0; kt < nk; ++kt) {
        const int st = kt & 1;
        store(st);
        __syncthreads();
        if (kt + 1 < nk) load((kt + 1) * LBK);
#pragma unroll
        for (int kk = 0; kk < LBK / 4; ++kk) {
            const int kr = 4 * kk + (l >> 4);
            ACC fa[4], fb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) fa[a] = As[st][kr][64 * wm + 16 * a + (l & 15)];
#pragma unroll
            for (int b = 0; b < 4; ++b) fb[b] = Bs[st][kr][64 * wn + 16 * b + (l & 15)];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma16<ACC>::op(fb[b], fa[a], acc[a][b]);
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + 64 * wm + 16 * a + (l & 15);
                const int j = col0 + 64 * wn + 16 * b + mfma16<ACC>::orow(l, r);
                if (i < M && j < N) {
                    TC *p = C + (size_t)j * ldc + i;
                    const TC v = (TC)alpha * (TC)acc[a][b][r];
                    if (beta != ACC(0)) *p = v + (TC)beta * (*p);
                    else *p = v;
                }
            }
}

// ---------------------------------------------------------------- BF16 inputs
// Operands rounded to bfloat16 (round to nearest even) on their way into LDS
// and multiplied by v_mfma_f32_16x16x32_bf16 with binary32 accumulation.  A
// binary64 operand is rounded to binary32 first.  Products of two bf16
// values are exact in binary32, so the result equals the binary32 GEMM of
// the rounded operands up to the order of the binary32 additions.
SYLV_DEVINL unsigned short bf16_rne(float x) {
    unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// binary16 (round to nearest even by the hardware conversion; overflow to
// Inf, gradual underflow), the narrow format of the FP16 option
SYLV_DEVINL unsigned short fp16_rne(float x) {
    const _Float16 h = (_Float16)x;
    return __builtin_bit_cast(unsigned short, h);
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// narrow-operand formats of the GEMM-shaped updates
constexpr int NARROW_BF16 = 1, NARROW_FP16 = 2;

template <int FMT>
SYLV_DEVINL unsigned short narrow_rne(float x) {
    if constexpr (FMT == NARROW_FP16) return fp16_rne(x);
    else return bf16_rne(x);
}

// one 16x16x32 MFMA step on 8 narrow values per lane
template <int FMT>
SYLV_DEVINL f32x4 mfma_narrow(uint4 a, uint4 b, f32x4 c) {
    if constexpr (FMT == NARROW_FP16)
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                     0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      c, 0, 0, 0);
}
constexpr int HBK = 32, HLD = HBK + 8;  // K slab and LDS row length (ushort; 80-byte rows)

template <int FMT, typename TA, typename TB, typename TC>
SYLV_DEVINL void gemm_bf16_tile(int M, int N, int K, const TA *__restrict__ A, int lda, int ta,
                                const TB *__restrict__ B, int ldb, int tb, TC *__restrict__ C, int ldc,
                                double alpha, float beta, TB bscale, int row0, int col0,
                                unsigned short (&As)[GBM][HLD], unsigned short (&Bs)[GBN][HLD]) {
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wm = w & 1, wn = w >> 1;
    f32x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    // raw operands; rounded to the narrow format when the slab goes to LDS
    TA ra[8];
    TB rb[8];
    // slab element r of this thread: A (i, k) and B (k, j) with coalesced global reads
    auto aidx = [&](int r, int &i, int &k) {
        if (!ta) { i = t & 63; k = (t >> 6) + 4 * r; } else { k = t & 31; i = (t >> 5) + 8 * r; }
    };
    auto bidx = [&](int r, int &k, int &j) {
        if (!tb) { k = t & 31; j = (t >> 5) + 8 * r; } else { j = t & 63; k = (t >> 6) + 4 * r; }
    };
    auto load = [&](int k0) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            int i, k;
            aidx(r, i, k);
            const int gi = row0 + i, gk = k0 + k;
            TA v = TA(0);
            if (gi < M && gk < K) v = ta ? A[(size_t)gi * lda + gk] : A[(size_t)gk * lda + gi];
            ra[r] = v;
            int j;
            bidx(r, k, j);
            const int gj = col0 + j, gk2 = k0 + k;
            TB u = TB(0);
            if (gj < N && gk2 < K) u = tb ? B[(size_t)gk2 * ldb + gj] : B[(size_t)gj * ldb + gk2];
            rb[r] = u;
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            int i, k, j;
            aidx(r, i, k);
            As[i][k] = narrow_rne<FMT>((float)ra[r]);
            bidx(r, k, j);
            Bs[j][k] = narrow_rne<FMT>((float)(bscale * rb[r]));
        }
    };
    const int nk = (K + HBK - 1) / HBK;
    if (nk > 0) load(0);
    for (int kt = 0; kt < nk; ++kt) {
        store();
        __syncthreads();
        if (kt + 1 < nk) load((kt + 1) * HBK);
        const int kg = 8 * (l >> 4);
        uint4 fa[2], fb[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) fa[a] = *reinterpret_cast<const uint4 *>(&As[32 * wm + 16 * a + (l & 15)][kg]);
#pragma unroll
        for (int b = 0; b < 2; ++b) fb[b] = *reinterpret_cast<const uint4 *>(&Bs[32 * wn + 16 * b + (l & 15)][kg]);
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) acc[a][b] = mfma_narrow<FMT>(fb[b], fa[a], acc[a][b]);
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = row0 + 32 * wm + 16 * a + (l & 15);
                const int j = col0 + 32 * wn + 16 * b + mfma16<float>::orow(l, r);
                if (i < M && j < N) {
                    TC *p = C + (size_t)j * ldc + i;
                    const TC v = (TC)alpha * (TC)acc[a][b][r];
                    if (beta != 0.f) *p = v + (TC)beta * (*p);
                    else *p = v;
                }
            }
}

// Output tile of workgroup bid: all tiles column by column, or (upper = 1,
// square C) only the tiles on or above the diagonal, tm <= tn, in the order
// of sym_pair_index (the products whose result is known to be symmetric: the
// caller mirrors the upper triangle afterwards).
SYLV_DEVINL void tile_of(int bid, int tiles_m, int upper, int &tm, int &tn) {
    if (upper) sym_pair_index(bid, tm, tn);
    else {
        tm = bid % tiles_m;
        tn = bid / tiles_m;
    }
}

template <int FMT, typename TA, typename TB, typename TC>
__global__ __launch_bounds__(256) void gemm_bf16_kernel(int M, int N, int K, const TA *__restrict__ A,
                                                        int lda, int ta, const TB *__restrict__ B, int ldb,
                                                        int tb, TC *__restrict__ C, int ldc, double alpha,
                                                        float beta, int tiles_m, TB bscale, int upper) {
    __shared__ __align__(16) unsigned short As[GBM][HLD];
    __shared__ __align__(16) unsigned short Bs[GBN][HLD];
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    int tm, tn;
    tile_of(bid, tiles_m, upper, tm, tn);
    gemm_bf16_tile<FMT, TA, TB, TC>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, bscale, tm * GBM,
                                    tn * GBN, As, Bs);
}

template <typename TA, typename TB, typename TC, typename ACC>
__global__ __launch_bounds__(256) void gemm_kernel(int M, int N, int K,
                                                   const TA *__restrict__ A, int lda, int ta,
                                                   const TB *__restrict__ B, int ldb, int tb,
                                                   TC *__restrict__ C, int ldc, double alpha, ACC beta,
                                                   int tiles_m, TB bscale, int upper) {
    __shared__ ACC As[GBK][GBM + GPAD];
    __shared__ ACC Bs[GBK][GBN + GPAD];
    // XCD-aware tile order: consecutive workgroup ids go to different XCDs;
    // give each XCD a contiguous run of tiles (shares operand panels in L2).
    const int nblk = gridDim.x;
    int bid = blockIdx.x;
    if ((nblk & 7) == 0) bid = (bid & 7) * (nblk >> 3) + (bid >> 3);
    int tm, tn;
    tile_of(bid, tiles_m, upper, tm, tn);
    gemm_tile<TA, TB, TC, ACC>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, alpha, beta, bscale, tm * GBM,
                               tn * GBN, As, Bs);
}

// Split-K partial products for short, wide outputs (a panel of nb <= 64 rows
// times a long contraction: too few 64x64 tiles to fill the chip).  Slice z
// of the contraction, k in [z kc, min(K, (z + 1) kc)), writes its product
// op(A) op(B) to P + z M N (ld M); the caller sums the slices in order.
template <typename T>
__global__ __launch_bounds__(256) void gemm_splitk_kernel(int M, int N, int K, int kc,
                                                          const T *__restrict__ A, int lda, int ta,
                                                          const T *__restrict__ B, int ldb, int tb,
                                                          T *__restrict__ P, int tiles_m) {
    __shared__ T As[GBK][GBM + GPAD];
    __shared__ T Bs[GBK][GBN + GPAD];
    const int z = blockIdx.y, kb = z * kc;
    const int kl = min(kc, K - kb);
    const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
    const T *Az = ta ? A + kb : A + (size_t)kb * lda;
    const T *Bz = tb ? B + (size_t)kb * ldb : B + kb;
    gemm_tile<T, T, T, T>(M, N, kl, Az, lda, ta, Bz, ldb, tb, P + (size_t)z * M * N, M, 1.0, T(0), T(1),
                          tm * GBM, tn * GBN, As, Bs);
}

template <typename T>
int gemm_splitk(hipStream_t s, int ta, int tb, int M, int N, int K, const T *A, int lda, const T *B, int ldb,
                T *P, int ksplit) {
    if (M <= 0 || N <= 0 || K <= 0 || ksplit < 1) return 0;
    const int per = (K + ksplit - 1) / ksplit;
    const int kc = (per + GBK - 1) / GBK * GBK;
    const int nz = (K + kc - 1) / kc;   // every slice non-empty
    const int tm = (M + GBM - 1) / GBM, tn = (N + GBN - 1) / GBN;
    prof_add_work(KID_GEMM, 2.0 * M * N * K);
    ProfScope ps(KID_GEMM, s);
    hipLaunchKernelGGL((gemm_splitk_kernel<T>), dim3(tm * tn, nz), dim3(256), 0, s, M, N, K, kc, A, lda, ta, B,
                       ldb, tb, P, tm);
    return nz;
}
template int gemm_splitk<float>(hipStream_t, int, int, int, int, int, const float *, int, const float *, int,
                                float *, int);
template int gemm_splitk<double>(hipStream_t, int, int, int, int, int, const double *, int, const double *, int,
                                 double *, int);

// Batched form over the equations of a batch: grid.y = equation slot (in
// the order given), grid.x = 64x64 tile of that equation's n x n product.
// Operands are fields of the per-equation descriptor.
template <typename TA, typename TB, typename TC, typename ACC, int BF16IN>
__global__ __launch_bounds__(256) void gemm_batched_kernel(const BatchEq *__restrict__ eqs,
                                                           const int *__restrict__ order, int fa,
                                                           int ta, int fb, int tb, int fc,
                                                           double alpha, int amode, ACC beta) {
    typedef typename std::conditional<BF16IN != 0, unsigned short, ACC>::type LT;
    constexpr int R0 = BF16IN ? GBM : GBK, C0 = BF16IN ? HLD : GBM + GPAD;
    constexpr int C1 = BF16IN ? HLD : GBN + GPAD;
    __shared__ __align__(16) LT As[R0][C0];
    __shared__ __align__(16) LT Bs[BF16IN ? GBN : GBK][C1];
    const BatchEq &q = eqs[order[blockIdx.y]];
    if (!q.active) return;
    if ((amode & 4) && q.sym) return;    // product not needed by the symmetric specialisation
    if ((amode & 16) && !q.sym) return;  // product of the symmetric specialisation only
    // per-equation operand format under the learned selector: bit 32 takes
    // only the equations with narrow operands, bit 64 only the others
    if ((amode & 32) && q.narrow == 0) return;
    if ((amode & 64) && q.narrow != 0) return;
    const int n = q.n;
    const int tl = (n + GBM - 1) / GBM;
    if ((int)blockIdx.x >= tl * tl) return;
    const int tm = blockIdx.x % tl, tn = blockIdx.x / tl;
    // amode & 8: a symmetric result of a symmetric equation, only the tiles
    // on or above the diagonal (the caller mirrors them)
    if ((amode & 8) && q.sym && tm > tn) return;
    // amode & 3 == 1 scales op(B) by scale_e before the conversion to ACC (a
    // binary64 residual brought to unit size ahead of the binary32 cast);
    // == 2 multiplies the product by 1 / scale_e; amode & 4 skips equations
    // with the symmetric flag
    double al = alpha;
    TB bs = TB(1);
    if ((amode & 3) == 1) bs = (TB)q.scale;
    else if ((amode & 3) == 2) al = alpha / q.scale;
    if constexpr (BF16IN != 0)
        gemm_bf16_tile<BF16IN, TA, TB, TC>(n, n, n, (const TA *)q.ptr[fa], q.ld[fa], ta, (const TB *)q.ptr[fb],
                                   q.ld[fb], tb, (TC *)q.ptr[fc], q.ld[fc], al, (float)beta, bs,
                                   tm * GBM, tn * GBN, As, Bs);
    else
        gemm_tile<TA, TB, TC, ACC>(n, n, n, (const TA *)q.ptr[fa], q.ld[fa], ta, (const TB *)q.ptr[fb],
                                   q.ld[fb], tb, (TC *)q.ptr[fc], q.ld[fc], al, beta, bs, tm * GBM,
                                   tn * GBN, As, Bs);
}

template <typename TA, typename TB, typename TC, typename ACC>
void gemm_batched(hipStream_t s, const BatchEq *eqs, const int *order, int batch, int nmax, int fa,
                  int ta, int fb, int tb, int fc, double alpha, int amode, ACC beta, int in_bf16) {
    if (batch <= 0) return;
    const int tl = (nmax + GBM - 1) / GBM;
    ProfScope ps(KID_BGEMM, s);
    if constexpr (sizeof(ACC) == sizeof(float)) {
        if (in_bf16 == NARROW_FP16) {
            hipLaunchKernelGGL((gemm_batched_kernel<TA, TB, TC, ACC, NARROW_FP16>), dim3(tl * tl, batch), dim3(256),
                               0, s, eqs, order, fa, ta, fb, tb, fc, alpha, amode, beta);
            return;
        }
        if (in_bf16) {
            hipLaunchKernelGGL((gemm_batched_kernel<TA, TB, TC, ACC, NARROW_BF16>), dim3(tl * tl, batch), dim3(256),
                               0, s, eqs, order, fa, ta, fb, tb, fc, alpha, amode, beta);
            return;
        }
    }
    hipLaunchKernelGGL((gemm_batched_kernel<TA, TB, TC, ACC, 0>), dim3(tl * tl, batch), dim3(256), 0, s,
                       eqs, order, fa, ta, fb, tb, fc, alpha, amode, beta);
}
template void gemm_batched<double, double, double, double>(hipStream_t, const BatchEq *, const int *,
                                                           int, int, int, int, int, int, int, double,
                                                           int, double, int);
template void gemm_batched<float, float, float, float>(hipStream_t, const BatchEq *, const int *, int,
                                                       int, int, int, int, int, int, double, int, float,
                                                       int);
template void gemm_batched<float, double, float, float>(hipStream_t, const BatchEq *, const int *, int,
                                                        int, int, int, int, int, int, double, int, float,
                                                        int);
template void gemm_batched<float, float, double, float>(hipStream_t, const BatchEq *, const int *, int,
                                                        int, int, int, int, int, int, double, int, float,
                                                        int);

// 128 x 128 tiles for large products (SYLV_GEMM128=0 in the environment
// keeps every product on the 64 x 64 kernel)
static const bool g_gemm128 = [] {
    const char *v = std::getenv("SYLV_GEMM128");
    return !(v && v[0] == '0');
}();

template <typename TA, typename TB, typename TC, typename ACC>
void gemm(hipStream_t s, int ta, int tb, int M, int N, int K, double alpha, const TA *A, int lda,
          const TB *B, int ldb, ACC beta, TC *C, int ldc, TB bscale, int in_bf16, int upper) {
    if (M <= 0 || N <= 0) return;
    int tm = (M + GBM - 1) / GBM, tn = (N + GBN - 1) / GBN;
    if (M != N || tm != tn) upper = 0;
    const int ntiles = upper ? tm * (tm + 1) / 2 : tm * tn;
    prof_add_work(KID_GEMM, upper ? 1.0 * M * (N + GBN) * K : 2.0 * M * N * K);
    ProfScope ps(KID_GEMM, s);
    if constexpr (sizeof(ACC) == sizeof(float)) {
        if (in_bf16 == NARROW_FP16) {
            hipLaunchKernelGGL((gemm_bf16_kernel<NARROW_FP16, TA, TB, TC>), dim3(ntiles), dim3(256), 0, s, M, N, K,
                               A, lda, ta, B, ldb, tb, C, ldc, alpha, (float)beta, tm, bscale, upper);
            return;
        }
        if (in_bf16) {
            hipLaunchKernelGGL((gemm_bf16_kernel<NARROW_BF16, TA, TB, TC>), dim3(ntiles), dim3(256), 0, s, M, N, K,
                               A, lda, ta, B, ldb, tb, C, ldc, alpha, (float)beta, tm, bscale, upper);
            return;
        }
    }
    // the 128-wide tile pays off on long contractions over enough tiles to
    // fill the chip; the Hessenberg's panel-width products (K = 32) run
    // faster on the 64-wide tile (four times the workgroups)
    if (M >= LBM && N >= LBM && K >= 256 && (M / LBM) * (N / LBM) >= 64 && g_gemm128) {
        const int tm2 = (M + LBM - 1) / LBM, tn2 = (N + LBM - 1) / LBM;
        const int up2 = (upper && tm2 == tn2) ? 1 : 0;
        const int nt2 = up2 ? tm2 * (tm2 + 1) / 2 : tm2 * tn2;
        // the transposes are template arguments: the LDS stores and global
        // loads of each operand layout compile without per-element branches
#define SYLV_G128(TAT, TBT)                                                                                     \
    hipLaunchKernelGGL((gemm128_kernel<TA, TB, TC, ACC, TAT, TBT>), dim3(nt2), dim3(256), 0, s, M, N, K, A, lda, B, \
                       ldb, C, ldc, alpha, beta, tm2, bscale, up2)
        if (!ta && !tb) SYLV_G128(0, 0);
        else if (ta && !tb) SYLV_G128(1, 0);
        else if (!ta) SYLV_G128(0, 1);
        else SYLV_G128(1, 1);
#undef SYLV_G128
        return;
    }
    hipLaunchKernelGGL((gemm_kernel<TA, TB, TC, ACC>), dim3(ntiles), dim3(256), 0, s, M, N, K, A,
                       lda, ta, B, ldb, tb, C, ldc, alpha, beta, tm, bscale, upper);
}

template void gemm<double, double, double, double>(hipStream_t, int, int, int, int, int, double,
                                                   const double *, int, const double *, int,
                                                   double, double *, int, double, int, int);
template void gemm<float, double, double, double>(hipStream_t, int, int, int, int, int, double,
                                                  const float *, int, const double *, int, double,
                                                  double *, int, double, int, int);
template void gemm<float, float, float, float>(hipStream_t, int, int, int, int, int, double,
                                               const float *, int, const float *, int, float,
                                               float *, int, float, int, int);
template void gemm<float, double, float, float>(hipStream_t, int, int, int, int, int, double,
                                                const float *, int, const double *, int, float,
                                                float *, int, double, int, int);
template void gemm<float, float, double, float>(hipStream_t, int, int, int, int, int, double,
                                                const float *, int, const float *, int, float,
                                                double *, int, float, int, int);

}  // namespace sylv
