// Tuning constants and entry points of the Schur driver.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace sylv {

// NSMALL: largest active block finished by one full-window LDS kernel
//         (bounded by 160 KiB of LDS: two NSMALL^2 matrices);
// NW:     aggressive-early-deflation window;
// NB:     bulges per multishift sweep (2*NB shifts); ADV: rows a bulge chain
//         advances per LDS window phase (window <= ADV + 3*NB + 1);
// HNB/HS: Hessenberg panel width and GEMV column slices.
template <typename T> struct SchurParams;
template <> struct SchurParams<float> {
    static constexpr int NSMALL = 140, NW = 96, NB = 24, ADV = 48, HNB = 32, HS = 32;
};
template <> struct SchurParams<double> {
    static constexpr int NSMALL = 98, NW = 80, NB = 16, ADV = 40, HNB = 32, HS = 32;
};

template <typename T>
size_t schur_work_bytes(int n);

// H (n x n, ldh): in = A, out = T (real Schur form).  U (ldu): out = Schur
// vectors.  ws: schur_work_bytes(n) device bytes; hbuf: >= 8 KiB pinned host
// memory.  *qr_status = 1 if the iteration cap was hit.  Synchronises s.
template <typename T>
int schur_run(hipStream_t s, int n, T *H, int ldh, T *U, int ldu, char *ws, char *hbuf,
              int *qr_status, int bf16 = 0);

}  // namespace sylv
