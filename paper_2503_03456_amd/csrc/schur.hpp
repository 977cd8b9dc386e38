// Tuning constants and entry points of the Schur driver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace sylv {

// Tunables of the QR phase (runtime, per precision):
//   nsmall: largest active block finished by one full-window LDS kernel;
//   nw:     aggressive-early-deflation window;
//   nb:     bulges per multishift sweep (2 nb shifts);
//   adv:    rows a bulge chain advances per LDS window phase (the phase
//           window is <= adv + 3 nb + 1 rows);
//   nibble: skip the sweep when AED deflated more than nibble% of the window;
//   aedw:   waves of the AED kernel (4 or 7);
//   chasew: waves of the bulge-chase kernel (8 or 16);
//   chains: bulge chains a sweep's bulges are split into (1..4), chased in
//           disjoint windows by one workgroup each.
struct SchurTune {
    int nsmall, nw, nb, adv, nibble, aedw, chasew, chains;
};
// Compile-time bounds that size the workspace and keep every LDS window
// within 160 KiB: two nsmall^2 matrices, a phase window of <= WMAX rows.
template <typename T> struct SchurCaps;
template <> struct SchurCaps<float> {
    static constexpr int NSMALL = 140, WMAX = 141, NBMAX = 44, HNB = 32, HS = 16;
};
template <> struct SchurCaps<double> {
    static constexpr int NSMALL = 98, WMAX = 99, NBMAX = 32, HNB = 32, HS = 16;
};
template <typename T> SchurTune schur_tune();
// Validates against the bounds; returns 0 or -1.
template <typename T> int schur_tune_set(const SchurTune &t);

template <typename T>
size_t schur_work_bytes(int n);

// Pinned host staging the driver uses: control words, AED shift candidates
// and exceptional-shift data below 8 KiB, then up to 3 NBMAX staged shifts
// (3 values per bulge) from byte 8192 on.
template <typename T>
constexpr size_t schur_hbuf_bytes() {
    return 8192 + 3 * (size_t)SchurCaps<T>::NBMAX * sizeof(T);
}

// H (n x n, ldh): in = A, out = T (real Schur form).  U (ldu): out = Schur
// vectors.  ws: schur_work_bytes(n) device bytes; hbuf: at least
// schur_hbuf_bytes<T>() bytes of pinned host memory.  *qr_status = 1 if the
// iteration cap was hit.  Synchronises s.
template <typename T>
int schur_run(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, char *ws, char *hbuf,
              int *qr_status, int bf16 = 0);

}  // namespace sylv
