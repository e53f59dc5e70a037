// The handle of a reduced system and library-internal helpers shared by
// the solve path and the serving layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <vector>

#include "shiftsolve.h"

struct shs_handle {
    int64_t n = 0, m = 0, p = 0;
    int device = 0;
    int64_t ldh = 0;
    double *H = nullptr;       // n x n, sign-normalised m-Hessenberg
    float *H32 = nullptr;      // FP32 copy for the mixed-precision sweep
    double *Bw = nullptr;      // n x m, R = Q^T B (rows >= m zero)
    double *Rtop = nullptr;    // m x m leading block of R (ld m)
    double *rcolmax = nullptr; // max_i |R(i, c)|
    double *Ct = nullptr;      // p x n, C Q (ld max(1,p))
    int64_t ldct = 1;
    double *V = nullptr;       // Householder vectors: column j holds reflector j from row start[j]
    double *tauv = nullptr;    // n taus (reflectors 0..m-1 of Q_B, then m.. of Q_A)
    int64_t nrefl = 0;
    double *sgn = nullptr;     // diagonal signs
    double *offrow = nullptr;  // off-diagonal row sums of |H|
    double *diag = nullptr;    // diagonal of H
    double reduce_ms = 0.0;
    size_t resident = 0;
    // phase timing of the last solve (events recorded on the solve's stream)
    bool timing = false;
    struct Mark { int phase; int64_t shifts; hipEvent_t a, b; };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> pool;
    bool last_mixed = false;   // the last timed solve ran the mixed mode
    double tile_flops = 0.0, update_flops = 0.0;   // algorithmic flops of the blocked sweep's launches
    long long *dstats = nullptr;   // device counters of the mixed mode's last timed solve (3 values)
    // transposed systems: Ht = J H^T J (J the order-reversing permutation) is
    // upper m-Hessenberg; built on the first transposed solve
    double *Ht = nullptr, *ht_offrow = nullptr, *ht_diag = nullptr;
    hipEvent_t ht_ready = nullptr;
    std::mutex ht_mu;
};

enum { PH_SWEEP = 0, PH_QSTAR, PH_RESIDUAL, PH_SWEEP32, PH_SWEEP32D, PH_OTHER, PH_TILE, PH_UPDATE, PH_COUNT };

namespace shs {

// Variants of the certification (all fields optional): another matrix of the
// same order and band (with its off-diagonal row sums and diagonal for
// ||M - sigma I||_inf), nc solution columns per shift instead of m, and dense
// complex right-hand sides E (column sid nc + c at E + col lde * 2) instead
// of [R; 0], with a per-column scratch emax for their maxima.
struct CertifyOpts {
    const double *H = nullptr;
    const double *offrow = nullptr, *diag = nullptr;
    int nc = 0;
    const double *E = nullptr;
    int64_t lde = 0;
    unsigned long long *emax = nullptr;
};

// FP64 residual R - (H X - sigma X) and backward error of the listed shifts
// (dlist == nullptr: shifts 0 .. s_list-1; dcount set: the list's length is
// read on the device, s_list is then an upper bound); Res optional;
// resmax/xmax are per-column scratch of m * s_total entries.
hipError_t certify(shs_handle *h, int64_t s_list, const int32_t *dlist, const int *dcount, const double *shifts,
                   const double *X, int64_t ldx, double *Res, unsigned long long *resmax, unsigned long long *xmax,
                   double *eta, int32_t *status, int64_t s_total, double *Xt, hipStream_t st,
                   const CertifyOpts *opt = nullptr);

// Zero `bytes` bytes (a multiple of 8) at p with a kernel on st: the solve
// path clears its scratch this way rather than with hipMemsetAsync, so a
// solve can be recorded into a HIP graph and replayed.
hipError_t zero_fill(void *p, size_t bytes, hipStream_t st);

// C = alpha op(A) op(B) (+ C when accumulate) on the FP64 matrix cores, for
// other translation units (the GEMM kernels are instantiated once, in the
// unit of the reduction); part (part_elems doubles, may be null) is the
// split-K workspace.
hipError_t dgemm(bool ta, bool tb, int M, int N, int K, double alpha, const double *A, int64_t lda, const double *B,
                 int64_t ldb, double *C, int64_t ldc, bool accumulate, double *part, size_t part_elems,
                 hipStream_t st);

// G(:, j*m + c) = Ct X(:, j*m + c) for shifts 0 .. s-1.
hipError_t g_eval(shs_handle *h, int64_t s, const double *X, int64_t ldx, double *G, int64_t ldg, hipStream_t st);

}  // namespace shs
