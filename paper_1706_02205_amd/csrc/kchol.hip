// HIP kernels (gfx950) and the C ABI of the sparse-Cholesky library.
//
// Data layout in HBM (one factor, carved from a caller-owned workspace):
//   xh       N x d f64   points in maximin order
//   colptr   (N+1) i64, rowidx nnz i32        pattern S by columns (CSC)
//   rowptr   (N+1) i64, colidx nnz i32        the same entries by rows (CSR)
//   csc2csr  nnz u32                          CSR position of each CSC entry
//   L        nnz f64 (FP64) | nnz f32 + N f64 diagonal (MIXED), stored by rows
//   units    64-entry column chunks grouped by DAG level
// L is stored by rows because the factorization reads rows (left-looking,
// see ichol_level) far more often than it writes columns.
//
// Compiled with -ffp-contract=off: every fused multiply-add is written out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "crmath.h"
#include "plan.h"

using kc::Unit;

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;                    // 4 wavefronts
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int64_t kLongColumn = 4096;          // backward solve: longer columns use a whole wavefront
constexpr int kMaxRhsPerPass = 8;

enum Counter { kNonpos = 0, kShifted = 1, kUpdates = 2, kExpHard = 3, kNumCounters = 8 };

// ---------------------------------------------------------------------------
// small kernels
__global__ void zero_u64(unsigned long long* p, int n) {
    int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

__global__ void gather_points(const double* __restrict__ x, const int32_t* __restrict__ perm, int64_t n, int d,
                              double* __restrict__ xh) {
    int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n * d) return;
    int64_t k = i / d;
    int t = int(i - k * d);
    xh[i] = x[int64_t(perm[k]) * d + t];
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// ---------------------------------------------------------------------------
// A1: Theta on S in CSC order, one wavefront per 64-entry column chunk.
template <int TWONU>
__global__ __launch_bounds__(kBlock) void theta_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                       const int64_t* __restrict__ colptr,
                                                       const int32_t* __restrict__ rowidx,
                                                       const double* __restrict__ xh, int d, double ell,
                                                       double* __restrict__ theta,
                                                       unsigned long long* __restrict__ counters) {
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= nunits) return;
    int lane = threadIdx.x % kWave;
    int j = __builtin_amdgcn_readfirstlane(units[u].col);
    int first = __builtin_amdgcn_readfirstlane(units[u].first);
    int64_t e = colptr[j] + first + lane;
    if (e >= colptr[j + 1]) return;
    int k = rowidx[e];
    int hard = 0;
    double r = kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d);
    theta[e] = kcdev::matern<TWONU>(r, ell, hard);
    if (hard) atomicAdd(counters + kExpHard, 1ull);
}

// ---------------------------------------------------------------------------
// A1+A2 (FP64): Theta on S fused into ICHOL(0), one DAG level per launch.
//
// Left-looking form of the paper's incomplete Cholesky: entry (k,j) of column j
// starts at Theta_kj and receives, for every parent i < j with (j,i) and (k,i)
// in S, in ascending i, the update A_kj <- fma(-L_ki, L_ji, A_kj) -- the same
// operations in the same order as the right-looking algorithm of Section 2.2,
// so the result is bitwise that algorithm's.  All parents of column j lie in
// earlier levels, so a level's columns are independent.
//
// One wavefront handles 64 consecutive entries of one column (a Unit); every
// lane owns one entry k.  The wave walks row j's parents (uniform across the
// wave) while each lane advances a cursor along row k of L (stored by rows), so
// the matching L_ki is found by a merge of two ascending lists without search.
// The pivot A_jj is accumulated uniformly by every wave of column j from row j,
// so chunks of a long column need no inter-wave communication.
template <int TWONU, bool COUNT>
__global__ __launch_bounds__(kBlock) void ichol_f64(const Unit* __restrict__ units, int64_t ubeg, int64_t uend,
                                                    const int64_t* __restrict__ colptr,
                                                    const int32_t* __restrict__ rowidx,
                                                    const uint32_t* __restrict__ csc2csr,
                                                    const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colidx, double* __restrict__ Lv,
                                                    const double* __restrict__ xh, int d, double ell, int policy,
                                                    double tau, unsigned long long* __restrict__ counters) {
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int64_t u = ubeg + int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= uend) return;
    int lane = threadIdx.x % kWave;
    int j = __builtin_amdgcn_readfirstlane(units[u].col);
    int first = __builtin_amdgcn_readfirstlane(units[u].first);
    int64_t c1 = colptr[j + 1];
    int64_t e = colptr[j] + first + lane;
    bool active = e < c1;
    int k = active ? rowidx[e] : j;

    int hard = 0;
    double acc = kcdev::matern<TWONU>(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d), ell, hard);
    double dacc = 1.0;  // Theta_jj

    int64_t t0 = rowptr[j], t1 = rowptr[j + 1] - 1;  // parents of j (the diagonal is last)
    int64_t p = rowptr[k];
    int ci = colidx[p];
    unsigned long long hits = 0;
    for (int64_t t = t0; t < t1; ++t) {
        int i = colidx[t];
        double lji = Lv[t];
        dacc = __builtin_fma(-lji, lji, dacc);
        while (ci < i) ci = colidx[++p];
        if (ci == i) {
            acc = __builtin_fma(-Lv[p], lji, acc);
            if (COUNT && lji != 0.0) ++hits;
        }
    }

    bool zero = false, shifted = false;
    double piv = dacc;
    if (policy == KC_PIVOT_ZERO) {
        zero = !(piv > 0.0);
    } else {
        double fl = tau * 1.0;
        if (!(piv > fl)) {
            piv = fl;
            shifted = true;
        }
    }
    double ljj = zero ? 0.0 : __builtin_sqrt(piv);
    if (active) Lv[csc2csr[e]] = zero ? 0.0 : (k == j ? ljj : acc / ljj);

    if (first == 0 && lane == 0) {
        if (zero) atomicAdd(counters + kNonpos, 1ull);
        if (shifted) atomicAdd(counters + kShifted, 1ull);
    }
    if (COUNT) {
        unsigned long long tot = wave_sum(active ? hits : 0ull);
        if (lane == 0 && tot) atomicAdd(counters + kUpdates, tot);
    }
    if (hard && active) atomicAdd(counters + kExpHard, 1ull);
}

// A1+A2 (MIXED): off-diagonal Theta, updates and stored L in FP32; the pivot is
// accumulated in FP64 from exact FP32 x FP32 products; sqrt and division in FP64.
template <int TWONU, bool COUNT>
__global__ __launch_bounds__(kBlock) void ichol_mixed(const Unit* __restrict__ units, int64_t ubeg, int64_t uend,
                                                      const int64_t* __restrict__ colptr,
                                                      const int32_t* __restrict__ rowidx,
                                                      const uint32_t* __restrict__ csc2csr,
                                                      const int64_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colidx, float* __restrict__ Lf,
                                                      double* __restrict__ diag, const double* __restrict__ xh, int d,
                                                      double ell, int policy, double tau,
                                                      unsigned long long* __restrict__ counters) {
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int64_t u = ubeg + int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= uend) return;
    int lane = threadIdx.x % kWave;
    int j = __builtin_amdgcn_readfirstlane(units[u].col);
    int first = __builtin_amdgcn_readfirstlane(units[u].first);
    int64_t c1 = colptr[j + 1];
    int64_t e = colptr[j] + first + lane;
    bool active = e < c1;
    int k = active ? rowidx[e] : j;

    float r = float(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d));
    float acc = kcdev::matern_f32<TWONU>(r, float(ell));
    double dacc = 1.0;

    int64_t t0 = rowptr[j], t1 = rowptr[j + 1] - 1;
    int64_t p = rowptr[k];
    int ci = colidx[p];
    unsigned long long hits = 0;
    for (int64_t t = t0; t < t1; ++t) {
        int i = colidx[t];
        float lji = Lf[t];
        dacc = __builtin_fma(-double(lji), double(lji), dacc);
        while (ci < i) ci = colidx[++p];
        if (ci == i) {
            acc = __builtin_fmaf(-Lf[p], lji, acc);
            if (COUNT && lji != 0.0f) ++hits;
        }
    }

    bool zero = false, shifted = false;
    double piv = dacc;
    if (policy == KC_PIVOT_ZERO) {
        zero = !(piv > 0.0);
    } else {
        double fl = tau * 1.0;
        if (!(piv > fl)) {
            piv = fl;
            shifted = true;
        }
    }
    double ljj = zero ? 0.0 : __builtin_sqrt(piv);
    if (active) {
        float out = zero ? 0.0f : (k == j ? float(ljj) : float(double(acc) / ljj));
        Lf[csc2csr[e]] = out;
        if (k == j) diag[j] = ljj;
    }
    if (first == 0 && lane == 0) {
        if (zero) atomicAdd(counters + kNonpos, 1ull);
        if (shifted) atomicAdd(counters + kShifted, 1ull);
    }
    if (COUNT) {
        unsigned long long tot = wave_sum(active ? hits : 0ull);
        if (lane == 0 && tot) atomicAdd(counters + kUpdates, tot);
    }
}

// ---------------------------------------------------------------------------
// A3: y = L^{-1} P b by rows (forward levels), x = P^T L^{-T} y by columns
// (reverse levels).  Each row / short column is one lane that accumulates its
// right-hand sides in registers in ascending index order, exactly like the
// sequential substitution; long columns of the backward sweep use a whole
// wavefront with a fixed-order lane reduction.

template <typename VT>
__device__ __forceinline__ double diag_of(const VT* Lv, const double* diag, int64_t rowend, int k) {
    if constexpr (sizeof(VT) == 8) return Lv[rowend];
    else return diag[k];
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void fwd_solve(const int32_t* __restrict__ rows, int64_t beg, int64_t end,
                                                    const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ colidx, const VT* __restrict__ Lv,
                                                    const double* __restrict__ diag,
                                                    const int32_t* __restrict__ perm, const double* __restrict__ b,
                                                    int ld, int r0, double* __restrict__ y) {
    int64_t t = beg + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= end) return;
    int k = rows[t];
    double acc[NR];
    const double* bk = b + int64_t(perm[k]) * ld + r0;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = bk[r];
    int64_t p1 = rowptr[k + 1] - 1;
    for (int64_t p = rowptr[k]; p < p1; ++p) {
        double l = double(Lv[p]);
        const double* yi = y + int64_t(colidx[p]) * ld + r0;
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = __builtin_fma(-l, yi[r], acc[r]);
    }
    double lkk = diag_of(Lv, diag, p1, k);
    double* yk = y + int64_t(k) * ld + r0;
#pragma unroll
    for (int r = 0; r < NR; ++r) yk[r] = (lkk == 0.0) ? 0.0 : acc[r] / lkk;
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void bwd_solve_short(const int32_t* __restrict__ cols, int64_t beg, int64_t end,
                                                          const int64_t* __restrict__ colptr,
                                                          const int32_t* __restrict__ rowidx,
                                                          const uint32_t* __restrict__ csc2csr,
                                                          const VT* __restrict__ Lv, const double* __restrict__ diag,
                                                          const int32_t* __restrict__ perm, int ld, int r0,
                                                          double* __restrict__ y, double* __restrict__ x) {
    int64_t t = beg + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= end) return;
    int j = cols[t];
    double acc[NR];
    double* yj = y + int64_t(j) * ld + r0;
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = yj[r];
    int64_t c0 = colptr[j], c1 = colptr[j + 1];
    for (int64_t e = c0 + 1; e < c1; ++e) {
        double l = double(Lv[csc2csr[e]]);
        const double* xk = y + int64_t(rowidx[e]) * ld + r0;
#pragma unroll
        for (int r = 0; r < NR; ++r) acc[r] = __builtin_fma(-l, xk[r], acc[r]);
    }
    double ljj;
    if constexpr (sizeof(VT) == 8) ljj = Lv[csc2csr[c0]];
    else ljj = diag[j];
    double* xo = x + int64_t(perm[j]) * ld + r0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double v = (ljj == 0.0) ? 0.0 : acc[r] / ljj;
        yj[r] = v;
        xo[r] = v;
    }
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void bwd_solve_long(const int32_t* __restrict__ cols, int64_t beg, int64_t end,
                                                         const int64_t* __restrict__ colptr,
                                                         const int32_t* __restrict__ rowidx,
                                                         const uint32_t* __restrict__ csc2csr,
                                                         const VT* __restrict__ Lv, const double* __restrict__ diag,
                                                         const int32_t* __restrict__ perm, int ld, int r0,
                                                         double* __restrict__ y, double* __restrict__ x) {
    int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int64_t t = beg + int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (t >= end) return;
    int lane = threadIdx.x % kWave;
    int j = cols[t];
    int64_t c0 = colptr[j], c1 = colptr[j + 1];
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    for (int64_t e = c0 + 1 + lane; e < c1; e += kWave) {
        double l = double(Lv[csc2csr[e]]);
        const double* xk = y + int64_t(rowidx[e]) * ld + r0;
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] = __builtin_fma(l, xk[r], s[r]);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s[r] += __shfl_xor(s[r], off, kWave);
    if (lane == 0) {
        double ljj;
        if constexpr (sizeof(VT) == 8) ljj = Lv[csc2csr[c0]];
        else ljj = diag[j];
        double* yj = y + int64_t(j) * ld + r0;
        double* xo = x + int64_t(perm[j]) * ld + r0;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v = (ljj == 0.0) ? 0.0 : (yj[r] - s[r]) / ljj;
            yj[r] = v;
            xo[r] = v;
        }
    }
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

namespace kc {
static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
}  // namespace kc

#define KC_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t _e = (call);                                                                \
        if (_e != hipSuccess) {                                                                \
            kc::set_error(std::string(#call) + ": " + hipGetErrorString(_e));                  \
            return KC_EHIP;                                                                    \
        }                                                                                      \
    } while (0)

#define KC_LAUNCH_CHECK()                                                                      \
    do {                                                                                       \
        hipError_t _e = hipGetLastError();                                                     \
        if (_e != hipSuccess) {                                                                \
            kc::set_error(std::string("kernel launch: ") + hipGetErrorString(_e));             \
            return KC_EHIP;                                                                    \
        }                                                                                      \
    } while (0)

struct kc_factor {
    int64_t n = 0, nnz = 0, nunits = 0;
    int32_t d = 0;
    kc_prec prec = KC_FP64;
    // device regions
    unsigned long long* counters = nullptr;
    double* xh = nullptr;
    int32_t* perm = nullptr;
    int64_t* colptr = nullptr;
    int32_t* rowidx = nullptr;
    uint32_t* csc2csr = nullptr;
    int64_t* rowptr = nullptr;
    int32_t* colidx = nullptr;
    void* L = nullptr;        // double[nnz] or float[nnz]
    double* diag = nullptr;   // MIXED only
    Unit* units = nullptr;
    int32_t* fwd_rows = nullptr;
    int32_t* bwd_cols = nullptr;
    // host schedule
    std::vector<int64_t> unit_off, fwd_off;
    std::vector<int64_t> bwd_beg, bwd_mid, bwd_end;  // per reverse level: short [beg,mid), long [mid,end)
    bool factorized = false;
    bool counted = false;
    hipStream_t last = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct Layout {
    size_t counters, xh, perm, colptr, rowidx, csc2csr, rowptr, colidx, L, diag, units, fwd, bwd, total;
};

Layout layout_of(const kc::Plan& p, kc_prec prec) {
    Layout o{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t r = at;
        at = align256(at + bytes);
        return r;
    };
    const size_t n = size_t(p.n), nnz = size_t(p.nnz());
    o.counters = take(kNumCounters * sizeof(unsigned long long));
    o.xh = take(n * p.d * sizeof(double));
    o.perm = take(n * sizeof(int32_t));
    o.colptr = take((n + 1) * sizeof(int64_t));
    o.rowidx = take(nnz * sizeof(int32_t));
    o.csc2csr = take(nnz * sizeof(uint32_t));
    o.rowptr = take((n + 1) * sizeof(int64_t));
    o.colidx = take(nnz * sizeof(int32_t));
    o.L = take(nnz * (prec == KC_FP64 ? sizeof(double) : sizeof(float)));
    o.diag = take(prec == KC_FP64 ? 0 : n * sizeof(double));
    o.units = take(p.units.size() * sizeof(Unit));
    o.fwd = take(n * sizeof(int32_t));
    o.bwd = take(n * sizeof(int32_t));
    o.total = at;
    return o;
}

int twonu_of(double nu) {
    if (nu == 0.5) return 1;
    if (nu == 1.5) return 3;
    if (nu == 2.5) return 5;
    return 0;
}

unsigned grid_for(int64_t items, int per_block) { return unsigned((items + per_block - 1) / per_block); }

}  // namespace

namespace {
template <typename VT, int NR>
kc_status solve_pass(const kc_factor* f, const double* b, double* x, int ld, int r0, double* y, hipStream_t s) {
    const VT* Lv = static_cast<const VT*>(f->L);
    const size_t nl = f->fwd_off.size() - 1;
    for (size_t v = 0; v < nl; ++v) {
        int64_t rb = f->fwd_off[v], re = f->fwd_off[v + 1];
        if (re <= rb) continue;
        fwd_solve<VT, NR><<<grid_for(re - rb, kBlock), kBlock, 0, s>>>(f->fwd_rows, rb, re, f->rowptr, f->colidx, Lv,
                                                                        f->diag, f->perm, b, ld, r0, y);
        KC_LAUNCH_CHECK();
    }
    for (size_t v = 0; v < f->bwd_beg.size(); ++v) {
        int64_t cb = f->bwd_beg[v], cm = f->bwd_mid[v], ce = f->bwd_end[v];
        if (cm > cb) {
            bwd_solve_short<VT, NR><<<grid_for(cm - cb, kBlock), kBlock, 0, s>>>(
                f->bwd_cols, cb, cm, f->colptr, f->rowidx, f->csc2csr, Lv, f->diag, f->perm, ld, r0, y, x);
            KC_LAUNCH_CHECK();
        }
        if (ce > cm) {
            bwd_solve_long<VT, NR><<<grid_for(ce - cm, kWavesPerBlock), kBlock, 0, s>>>(
                f->bwd_cols, cm, ce, f->colptr, f->rowidx, f->csc2csr, Lv, f->diag, f->perm, ld, r0, y, x);
            KC_LAUNCH_CHECK();
        }
    }
    return KC_OK;
}

template <typename VT>
kc_status solve_typed(const kc_factor* f, const double* b, double* x, int nrhs, double* y, hipStream_t s) {
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerPass) {
        int nr = std::min(kMaxRhsPerPass, nrhs - r0);
        kc_status st;
        switch (nr) {
            case 1: st = solve_pass<VT, 1>(f, b, x, nrhs, r0, y, s); break;
            case 2: st = solve_pass<VT, 2>(f, b, x, nrhs, r0, y, s); break;
            case 3: st = solve_pass<VT, 3>(f, b, x, nrhs, r0, y, s); break;
            case 4: st = solve_pass<VT, 4>(f, b, x, nrhs, r0, y, s); break;
            case 5: st = solve_pass<VT, 5>(f, b, x, nrhs, r0, y, s); break;
            case 6: st = solve_pass<VT, 6>(f, b, x, nrhs, r0, y, s); break;
            case 7: st = solve_pass<VT, 7>(f, b, x, nrhs, r0, y, s); break;
            default: st = solve_pass<VT, 8>(f, b, x, nrhs, r0, y, s); break;
        }
        if (st != KC_OK) return st;
    }
    return KC_OK;
}
}  // namespace

extern "C" {

const char* kc_status_string(kc_status s) {
    switch (s) {
        case KC_OK: return "ok";
        case KC_EINVAL: return "invalid argument";
        case KC_ENOMEM: return "out of host memory";
        case KC_EWORKSPACE: return "workspace too small";
        case KC_EHIP: return "HIP runtime error";
        case KC_ESTATE: return "call out of order";
        case KC_ERANGE: return "problem too large for 32-bit entry positions";
    }
    return "unknown status";
}

const char* kc_last_error(void) { return kc::g_err.c_str(); }

int32_t kc_device_count(void) {
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) return 0;
    return c;
}

kc_status kc_analyze(const double* x, int64_t n, int32_t d, double rho, kc_rule rule, int32_t nthreads,
                     kc_plan** out) {
    if (!out) {
        kc::set_error("kc_analyze: out is NULL");
        return KC_EINVAL;
    }
    *out = nullptr;
    if (!x || n < 1 || d < 1 || !(rho > 0.0) || !std::isfinite(rho) || (rule != KC_RULE_MAX && rule != KC_RULE_MIN)) {
        kc::set_error("kc_analyze: need x != NULL, n >= 1, d >= 1, finite rho > 0, rule MAX or MIN");
        return KC_EINVAL;
    }
    if (n >= (int64_t(1) << 31)) {
        kc::set_error("kc_analyze: n must be below 2^31");
        return KC_ERANGE;
    }
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(x[i])) {
            kc::set_error("kc_analyze: non-finite coordinate");
            return KC_EINVAL;
        }
    kc_plan* plan = new (std::nothrow) kc_plan;
    if (!plan) return KC_ENOMEM;
    try {
        kc::Plan& p = plan->p;
        p.n = n;
        p.d = d;
        p.rho = rho;
        p.rule = rule;
        p.perm.resize(size_t(n));
        p.l.resize(size_t(n));
        auto t0 = std::chrono::steady_clock::now();
        kc::maximin_order(x, n, d, nthreads, p.perm.data(), p.l.data());
        auto t1 = std::chrono::steady_clock::now();
        p.xh.resize(size_t(n) * d);
        for (int64_t k = 0; k < n; ++k)
            for (int t = 0; t < d; ++t) p.xh[size_t(k) * d + t] = x[size_t(p.perm[k]) * d + t];
        kc::build_pattern(p, nthreads);
        if (p.nnz() >= (int64_t(1) << 32)) {
            delete plan;
            kc::set_error("kc_analyze: nnz(S) >= 2^32");
            return KC_ERANGE;
        }
        auto t2 = std::chrono::steady_clock::now();
        kc::build_schedule(p, nthreads);
        auto t3 = std::chrono::steady_clock::now();
        p.t_order = std::chrono::duration<double>(t1 - t0).count();
        p.t_pattern = std::chrono::duration<double>(t2 - t1).count();
        p.t_schedule = std::chrono::duration<double>(t3 - t2).count();
    } catch (const std::bad_alloc&) {
        delete plan;
        kc::set_error("kc_analyze: out of host memory");
        return KC_ENOMEM;
    }
    *out = plan;
    return KC_OK;
}

kc_status kc_plan_info(const kc_plan* plan, kc_plan_info_t* info) {
    if (!plan || !info) return KC_EINVAL;
    const kc::Plan& p = plan->p;
    info->n = p.n;
    info->d = p.d;
    info->rule = p.rule;
    info->rho = p.rho;
    info->nnz = p.nnz();
    info->max_col = p.max_col;
    info->max_row = p.max_row;
    info->nlevels = p.nlevels;
    info->nrlevels = p.nrlevels;
    info->nunits = int64_t(p.units.size());
    info->t_order_s = p.t_order;
    info->t_pattern_s = p.t_pattern;
    info->t_schedule_s = p.t_schedule;
    return KC_OK;
}

kc_status kc_plan_export(const kc_plan* plan, int32_t* perm, double* l, int64_t* colptr, int32_t* rowidx) {
    if (!plan) return KC_EINVAL;
    const kc::Plan& p = plan->p;
    if (perm) std::memcpy(perm, p.perm.data(), p.perm.size() * sizeof(int32_t));
    if (l) std::memcpy(l, p.l.data(), p.l.size() * sizeof(double));
    if (colptr) std::memcpy(colptr, p.colptr.data(), p.colptr.size() * sizeof(int64_t));
    if (rowidx) std::memcpy(rowidx, p.rowidx.data(), p.rowidx.size() * sizeof(int32_t));
    return KC_OK;
}

kc_status kc_plan_levels(const kc_plan* plan, int32_t* level) {
    if (!plan || !level) return KC_EINVAL;
    std::memcpy(level, plan->p.level.data(), plan->p.level.size() * sizeof(int32_t));
    return KC_OK;
}

void kc_plan_destroy(kc_plan* plan) { delete plan; }

kc_status kc_factor_bytes(const kc_plan* plan, kc_prec prec, size_t* bytes) {
    if (!plan || !bytes || (prec != KC_FP64 && prec != KC_MIXED)) return KC_EINVAL;
    *bytes = layout_of(plan->p, prec).total;
    return KC_OK;
}

kc_status kc_factor_create(const kc_plan* plan, kc_prec prec, void* ws_dev, size_t ws_bytes, void* stream,
                           kc_factor** out) {
    if (!out) return KC_EINVAL;
    *out = nullptr;
    if (!plan || !ws_dev || (prec != KC_FP64 && prec != KC_MIXED)) {
        kc::set_error("kc_factor_create: need plan, workspace and prec FP64 or MIXED");
        return KC_EINVAL;
    }
    const kc::Plan& p = plan->p;
    Layout o = layout_of(p, prec);
    if (ws_bytes < o.total) {
        kc::set_error("kc_factor_create: workspace holds " + std::to_string(ws_bytes) + " bytes, needs " +
                      std::to_string(o.total));
        return KC_EWORKSPACE;
    }
    if (reinterpret_cast<uintptr_t>(ws_dev) % 256) {
        kc::set_error("kc_factor_create: workspace must be 256-byte aligned");
        return KC_EINVAL;
    }
    std::unique_ptr<kc_factor> f(new (std::nothrow) kc_factor);
    if (!f) return KC_ENOMEM;
    char* base = static_cast<char*>(ws_dev);
    f->n = p.n;
    f->nnz = p.nnz();
    f->d = p.d;
    f->prec = prec;
    f->nunits = int64_t(p.units.size());
    f->counters = reinterpret_cast<unsigned long long*>(base + o.counters);
    f->xh = reinterpret_cast<double*>(base + o.xh);
    f->perm = reinterpret_cast<int32_t*>(base + o.perm);
    f->colptr = reinterpret_cast<int64_t*>(base + o.colptr);
    f->rowidx = reinterpret_cast<int32_t*>(base + o.rowidx);
    f->csc2csr = reinterpret_cast<uint32_t*>(base + o.csc2csr);
    f->rowptr = reinterpret_cast<int64_t*>(base + o.rowptr);
    f->colidx = reinterpret_cast<int32_t*>(base + o.colidx);
    f->L = base + o.L;
    f->diag = prec == KC_MIXED ? reinterpret_cast<double*>(base + o.diag) : nullptr;
    f->units = reinterpret_cast<Unit*>(base + o.units);
    f->fwd_rows = reinterpret_cast<int32_t*>(base + o.fwd);
    f->bwd_cols = reinterpret_cast<int32_t*>(base + o.bwd);
    f->unit_off = p.unit_off;
    f->fwd_off = p.fwd_off;

    // backward schedule: per reverse level, short columns then long columns
    std::vector<int32_t> bwd(size_t(p.n));
    f->bwd_beg.resize(size_t(p.nrlevels));
    f->bwd_mid.resize(size_t(p.nrlevels));
    f->bwd_end.resize(size_t(p.nrlevels));
    {
        int64_t w = 0;
        for (int32_t v = 0; v < p.nrlevels; ++v) {
            f->bwd_beg[v] = w;
            for (int64_t q = p.bwd_off[v]; q < p.bwd_off[v + 1]; ++q) {
                int32_t j = p.bwd_cols[q];
                if (p.colptr[j + 1] - p.colptr[j] <= kLongColumn) bwd[size_t(w++)] = j;
            }
            f->bwd_mid[v] = w;
            for (int64_t q = p.bwd_off[v]; q < p.bwd_off[v + 1]; ++q) {
                int32_t j = p.bwd_cols[q];
                if (p.colptr[j + 1] - p.colptr[j] > kLongColumn) bwd[size_t(w++)] = j;
            }
            f->bwd_end[v] = w;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = size_t(p.n), nnz = size_t(p.nnz());
    KC_HIP(hipMemcpyAsync(f->perm, p.perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->colptr, p.colptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->rowidx, p.rowidx.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->csc2csr, p.csc2csr.data(), nnz * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->rowptr, p.rowptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->colidx, p.colidx.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->units, p.units.data(), p.units.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->fwd_rows, p.fwd_rows.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->bwd_cols, bwd.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    // pageable sources: make sure the copies are done before the host vectors can go away
    KC_HIP(hipStreamSynchronize(s));
    f->last = s;
    *out = f.release();
    return KC_OK;
}

kc_status kc_factorize(kc_factor* f, const double* x_dev, kc_kernel kernel, kc_pivot pivot, double tau,
                       int32_t count_updates, void* stream) {
    if (!f || !x_dev) return KC_EINVAL;
    int tn = twonu_of(kernel.nu);
    if (!tn || !(kernel.lengthscale > 0.0) || !std::isfinite(kernel.lengthscale)) {
        kc::set_error("kc_factorize: nu must be 0.5, 1.5 or 2.5 and the lengthscale finite and positive");
        return KC_EINVAL;
    }
    if (pivot != KC_PIVOT_ZERO && pivot != KC_PIVOT_SHIFT) return KC_EINVAL;
    if (pivot == KC_PIVOT_SHIFT && !(tau > 0.0 && std::isfinite(tau))) {
        kc::set_error("kc_factorize: KC_PIVOT_SHIFT needs a finite tau > 0");
        return KC_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    zero_u64<<<1, 64, 0, s>>>(f->counters, kNumCounters);
    KC_LAUNCH_CHECK();
    gather_points<<<grid_for(f->n * f->d, kBlock), kBlock, 0, s>>>(x_dev, f->perm, f->n, f->d, f->xh);
    KC_LAUNCH_CHECK();
    const bool cnt = count_updates != 0;
    const double ell = kernel.lengthscale;
    const int pol = int(pivot);
    const size_t nl = f->unit_off.size() - 1;
    for (size_t v = 0; v < nl; ++v) {
        int64_t ub = f->unit_off[v], ue = f->unit_off[v + 1];
        if (ue <= ub) continue;
        dim3 grid(grid_for(ue - ub, kWavesPerBlock));
#define KC_ICHOL_ARGS_F64                                                                                   \
    f->units, ub, ue, f->colptr, f->rowidx, f->csc2csr, f->rowptr, f->colidx, static_cast<double*>(f->L), \
        f->xh, f->d, ell, pol, tau, f->counters
#define KC_ICHOL_ARGS_MIX                                                                                  \
    f->units, ub, ue, f->colptr, f->rowidx, f->csc2csr, f->rowptr, f->colidx, static_cast<float*>(f->L), \
        f->diag, f->xh, f->d, ell, pol, tau, f->counters
        if (f->prec == KC_FP64) {
            switch (tn * 2 + (cnt ? 1 : 0)) {
                case 2: ichol_f64<1, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
                case 3: ichol_f64<1, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
                case 6: ichol_f64<3, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
                case 7: ichol_f64<3, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
                case 10: ichol_f64<5, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
                default: ichol_f64<5, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_F64); break;
            }
        } else {
            switch (tn * 2 + (cnt ? 1 : 0)) {
                case 2: ichol_mixed<1, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
                case 3: ichol_mixed<1, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
                case 6: ichol_mixed<3, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
                case 7: ichol_mixed<3, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
                case 10: ichol_mixed<5, false><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
                default: ichol_mixed<5, true><<<grid, kBlock, 0, s>>>(KC_ICHOL_ARGS_MIX); break;
            }
        }
#undef KC_ICHOL_ARGS_F64
#undef KC_ICHOL_ARGS_MIX
        KC_LAUNCH_CHECK();
    }
    f->factorized = true;
    f->counted = cnt;
    f->last = s;
    return KC_OK;
}

kc_status kc_theta(kc_factor* f, const double* x_dev, kc_kernel kernel, double* theta_dev, void* stream) {
    if (!f || !x_dev || !theta_dev) return KC_EINVAL;
    int tn = twonu_of(kernel.nu);
    if (!tn || !(kernel.lengthscale > 0.0)) return KC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    zero_u64<<<1, 64, 0, s>>>(f->counters, kNumCounters);
    KC_LAUNCH_CHECK();
    gather_points<<<grid_for(f->n * f->d, kBlock), kBlock, 0, s>>>(x_dev, f->perm, f->n, f->d, f->xh);
    KC_LAUNCH_CHECK();
    if (f->nunits > 0) {
        dim3 grid(grid_for(f->nunits, kWavesPerBlock));
        double ell = kernel.lengthscale;
        if (tn == 1) theta_kernel<1><<<grid, kBlock, 0, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->xh, f->d, ell, theta_dev, f->counters);
        else if (tn == 3) theta_kernel<3><<<grid, kBlock, 0, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->xh, f->d, ell, theta_dev, f->counters);
        else theta_kernel<5><<<grid, kBlock, 0, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->xh, f->d, ell, theta_dev, f->counters);
        KC_LAUNCH_CHECK();
    }
    f->last = s;
    return KC_OK;
}

kc_status kc_solve_bytes(const kc_factor* f, int32_t nrhs, size_t* bytes) {
    if (!f || !bytes || nrhs < 1) return KC_EINVAL;
    *bytes = size_t(f->n) * size_t(nrhs) * sizeof(double);
    return KC_OK;
}


kc_status kc_solve(const kc_factor* f, const double* b_dev, double* x_dev, int32_t nrhs, void* scratch_dev,
                   size_t scratch_bytes, void* stream) {
    if (!f || !b_dev || !x_dev || !scratch_dev || nrhs < 1) return KC_EINVAL;
    if (b_dev == x_dev) {
        kc::set_error("kc_solve: b and x must not alias");
        return KC_EINVAL;
    }
    if (!f->factorized) {
        kc::set_error("kc_solve: factor has not been computed");
        return KC_ESTATE;
    }
    if (scratch_bytes < size_t(f->n) * size_t(nrhs) * sizeof(double)) {
        kc::set_error("kc_solve: scratch smaller than n*nrhs doubles");
        return KC_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* y = static_cast<double*>(scratch_dev);
    kc_status st = f->prec == KC_FP64 ? solve_typed<double>(f, b_dev, x_dev, nrhs, y, s)
                                      : solve_typed<float>(f, b_dev, x_dev, nrhs, y, s);
    const_cast<kc_factor*>(f)->last = s;
    return st;
}

kc_status kc_factor_stats(kc_factor* f, kc_factor_stats_t* st) {
    if (!f || !st) return KC_EINVAL;
    unsigned long long c[kNumCounters];
    KC_HIP(hipStreamSynchronize(f->last));
    KC_HIP(hipMemcpy(c, f->counters, sizeof(c), hipMemcpyDeviceToHost));
    st->nonpositive = int64_t(c[kNonpos]);
    st->shifted = int64_t(c[kShifted]);
    st->rank = f->n - int64_t(c[kNonpos]);
    st->updates = f->counted ? int64_t(c[kUpdates]) : -1;
    st->exp_hard = int64_t(c[kExpHard]);
    return KC_OK;
}

kc_status kc_factor_export_L(const kc_factor* f, double* vals) {
    if (!f || !vals) return KC_EINVAL;
    if (!f->factorized) return KC_ESTATE;
    KC_HIP(hipStreamSynchronize(f->last));
    const size_t nnz = size_t(f->nnz);
    std::vector<uint32_t> c2r(nnz);
    std::vector<int64_t> colptr(size_t(f->n) + 1);
    KC_HIP(hipMemcpy(c2r.data(), f->csc2csr, nnz * sizeof(uint32_t), hipMemcpyDeviceToHost));
    KC_HIP(hipMemcpy(colptr.data(), f->colptr, colptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    if (f->prec == KC_FP64) {
        std::vector<double> v(nnz);
        KC_HIP(hipMemcpy(v.data(), f->L, nnz * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < nnz; ++e) vals[e] = v[c2r[e]];
    } else {
        std::vector<float> v(nnz);
        std::vector<double> dg(size_t(f->n));
        KC_HIP(hipMemcpy(v.data(), f->L, nnz * sizeof(float), hipMemcpyDeviceToHost));
        KC_HIP(hipMemcpy(dg.data(), f->diag, dg.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < nnz; ++e) vals[e] = double(v[c2r[e]]);
        for (int64_t j = 0; j < f->n; ++j) vals[colptr[size_t(j)]] = dg[size_t(j)];
    }
    return KC_OK;
}

void kc_factor_destroy(kc_factor* f) { delete f; }

}  // extern "C"
