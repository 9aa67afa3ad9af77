// Dense covariance matvec and preconditioned conjugate gradients (gfx950).
//
// The sparse factor is used as a preconditioner for CG on the dense system
// Theta x = b (Section 4.3 suggests CG with the factor when the approximation
// alone is not accurate enough).  Each iteration needs one product with the
// dense N x N Theta, whose entries are generated on the fly: the work is N^2
// evaluations of the kernel (a square root and an exponential each), bound by
// the FP64 vector ALUs, not by memory.  The generated values are contracted
// with the right-hand sides on the matrix cores (FP64 MFMA), which leaves the
// vector ALUs with the kernel evaluations alone.
//
// All reductions (dot products) use a fixed grid and a fixed combination order,
// so results are reproducible run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "factor.h"
#include "kchol.h"
#include "plan.h"

namespace kc {
void set_error(const std::string& msg);
}

namespace {

constexpr int kRows = 256;       // rows (threads) per block
constexpr int kTileJ = 256;      // columns staged per LDS tile (at most)
constexpr int kDotBlocks = 512;  // fixed grid of the dot-product reduction

// exp(x) for -707 <= x <= 0 by table lookup and a short polynomial (Tang's
// method, ACM TOMS 15(2), 1989): x = (256 m + j) ln2/256 + r with
// |r| <= ln2/512, so exp(x) = 2^m 2^(j/256) exp(r).  2^(j/256) comes from a
// 256-entry table in LDS, exp(r) - 1 from its degree-4 Taylor polynomial
// (truncation below 4e-17).  The reduction uses ln2/256 rounded to double
// alone: the error that leaves in r is below 8e-17 a relative, about 4 ulp at
// a = 5, far below what the dense product needs.  On this range 2^m never
// leaves the normal numbers.
constexpr int kExpBits = 8;
constexpr int kExpSize = 1 << kExpBits;
constexpr double kShift = 6755399441055744.0;          // 1.5 * 2^52: adding it rounds to an integer
constexpr double kInvLn2xN = 369.32993046757463;       // 256 / ln 2 (only selects the reduction)
constexpr double kLn2dN = 0.0027076061740622863;       // ln 2 / 256 rounded to double
constexpr double kMaxArg = 707.0;                      // exp(-707) is still a normal number

struct ExpTable {
    double t[kExpSize];  // 2^(j/256)
};

ExpTable make_exp_table() {
    ExpTable e{};
    for (int j = 0; j < kExpSize; ++j)
        e.t[j] = static_cast<double>(std::exp2(static_cast<long double>(j) / static_cast<long double>(kExpSize)));
    return e;
}

// exp(-a) for 0 <= a <= kMaxArg; c6 is 1/6, held by the caller in a vector
// register (an fma can read one scalar constant, and 1/24 is the other).
__device__ __forceinline__ double exp_neg(double a, const double* __restrict__ tab, double c6) {
    const double x = -a;
    const double t = __builtin_fma(x, kInvLn2xN, kShift);
    const double kf = t - kShift;
    const int k = __double2loint(t);  // the low word holds the integer
    const double r = __builtin_fma(-kf, kLn2dN, x);
    double q = __builtin_fma(r, 1.0 / 24.0, c6);
    q = __builtin_fma(r, q, 0.5);
    q = __builtin_fma(r, q, 1.0);
    const double p = r * q;  // exp(r) - 1
    const double tj = tab[k & (kExpSize - 1)];
    return __builtin_amdgcn_ldexp(__builtin_fma(tj, p, tj), k >> kExpBits);
}

// sqrt(s) for s > 0 from the hardware reciprocal square root y (relative error
// about 5e-8) and one second-order correction: with g = s y and c = 1 - y g
// (one rounding), sqrt(s) = g (1 - c)^(-1/2) = g (1 + c/2 + 3c^2/8 + O(c^3));
// the rounding of g enters as half its relative error, so the result is within
// about one ulp.
__device__ __forceinline__ double sqrt_pos(double s) {
    const double y = __builtin_amdgcn_rsq(s);
    const double g = s * y;
    const double c = __builtin_fma(-y, g, 1.0);
    const double q = __builtin_fma(c, 0.375, 0.5);
    return __builtin_fma(g * c, q, g);
}

// Matern-nu/2 closed forms of Section 4.4 at a = c r / l (c = 1, sqrt 3,
// sqrt 5 for TWONU = 2 nu = 1, 3, 5).  a is capped at kMaxArg: beyond it every
// form is below 1e-300, and the cap replaces those entries by their value at
// the cap, an absolute change below 2e-302.
template <int TWONU>
__device__ __forceinline__ double matern_fast(double a, const double* __restrict__ tab, double c6) {
    a = fmin(a, kMaxArg);
    const double e = exp_neg(a, tab, c6);
    if constexpr (TWONU == 1) {
        return e;
    } else if constexpr (TWONU == 3) {
        return __builtin_fma(a, e, e);
    } else {
        return (1.0 + a + a * a * (1.0 / 3.0)) * e;
    }
}

// Y[i, r0+r] = sum_j Theta(x_i, x_j) X[j, r0+r].  x: n x d (any order, X and Y
// in the same order).  D = d for d <= 3 (coordinates in registers), D = 0 for
// any d <= 32 (own coordinates re-read through the cache).  Columns stream
// through LDS in tiles shared by the 256 rows of a block.
//
// The kernel values are generated on the vector ALUs; their contraction with
// the right-hand sides runs on the matrix cores, by v_mfma_f64_4x4x4f64: four independent 4 x 4 x 4 blocks per wave, lane
// l = 16 s + 4 q + t supplying A[q][t][s], B[q][s][t] and receiving D[q][s][t].
// A wave owns kGroups groups of 16 rows; in a group, block q covers rows
// 4q..4q+3.  For each quad of staged columns (column s of the quad), lane l
// evaluates Theta(row 4q + t, column s) on the vector ALUs; B[s][t] is
// X[column s][right-hand side t] (two instructions cover 8 right-hand sides,
// with no padding), and lane l ends with Y[row 4q + s][t].  The order of
// summation over j is fixed (by quads, ascending), so results are
// reproducible run to run.
constexpr int kGroups = 2;                    // 16-row groups per wave
constexpr int kMfmaRhs = 8;                   // right-hand sides per pass (two 4-wide blocks)
constexpr int kMfmaRows = 4 * 16 * kGroups;   // rows per block (4 waves)
constexpr int kMfmaLds = 65536;               // LDS bytes per block at most

template <int TWONU, int D, int NB>
__global__ __launch_bounds__(256) void dense_matvec_mfma(const double* __restrict__ x, int64_t n, int d,
                                                         double scale, const double* __restrict__ X, int ld,
                                                         int r0, int nr, double* __restrict__ Y, ExpTable et,
                                                         int tj) {
    extern __shared__ double tile[];  // kExpSize table entries, tj * d coordinates, tj * 8 values
    double* tab = tile;
    double* sx = tile + kExpSize;
    double* sv = sx + size_t(tj) * d;
    for (int q = threadIdx.x; q < kExpSize; q += blockDim.x) tab[q] = et.t[q];
    // With coordinates in registers (D > 0) both sides are multiplied by `scale`
    // as they are loaded, so the distance comes out as a = c r / l directly.
    const double cs = D > 0 ? scale : 1.0;
    double c6 = 1.0 / 6.0;
    asm volatile("" : "+v"(c6));  // kept in a vector register for the whole loop
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t4 = lane & 3, q4 = (lane >> 2) & 3, s4 = lane >> 4;
    const int64_t row_base = int64_t(blockIdx.x) * kMfmaRows + int64_t(wave) * 16 * kGroups;
    int64_t ic[kGroups];
    double xi[kGroups][D > 0 ? D : 1];
    double acc[kGroups][NB];
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const int64_t i = row_base + g * 16 + 4 * q4 + t4;
        ic[g] = i < n ? i : n - 1;
#pragma unroll
        for (int t = 0; t < (D > 0 ? D : 1); ++t) xi[g][t] = D > 0 ? x[ic[g] * D + t] * cs : 0.0;
#pragma unroll
        for (int b = 0; b < NB; ++b) acc[g][b] = 0.0;
    }
    for (int64_t j0 = 0; j0 < n; j0 += tj) {
        const int m = int(n - j0 < tj ? n - j0 : tj);
        const int mq = (m + 3) & ~3;  // whole quads; the padding columns carry zero weights
        for (int q = threadIdx.x; q < mq * d; q += 256) sx[q] = q < m * d ? x[j0 * d + q] * cs : 0.0;
        for (int q = threadIdx.x; q < mq * kMfmaRhs; q += 256) {
            const int jj = q >> 3, r = q & 7;
            sv[q] = (jj < m && r < nr) ? X[(j0 + jj) * ld + r0 + r] : 0.0;
        }
        __syncthreads();
        for (int jq = 0; jq < mq; jq += 4) {
            const int jj = jq + s4;
            double bv[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) bv[b] = sv[jj * kMfmaRhs + 4 * b + t4];
#pragma unroll
            for (int g = 0; g < kGroups; ++g) {
                // s starts at 1e-300 so that s = 0 (a point with itself) gives
                // a = 1e-150 (the kernel is 1 to the last bit) instead of 0 * inf
                double s = 1e-300;
                if constexpr (D > 0) {
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        const double df = xi[g][t] - sx[jj * D + t];
                        s = __builtin_fma(df, df, s);
                    }
                } else {
                    for (int t = 0; t < d; ++t) {
                        const double df = x[ic[g] * d + t] - sx[jj * d + t];
                        s = __builtin_fma(df, df, s);
                    }
                }
                const double th = matern_fast<TWONU>(D > 0 ? sqrt_pos(s) : sqrt_pos(s) * scale, tab, c6);
#pragma unroll
                for (int b = 0; b < NB; ++b) acc[g][b] = __builtin_amdgcn_mfma_f64_4x4x4f64(th, bv[b], acc[g][b], 0, 0, 0);
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int g = 0; g < kGroups; ++g) {
        const int64_t i = row_base + g * 16 + 4 * q4 + s4;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int r = 4 * b + t4;
            if (i < n && r < nr) Y[i * ld + r0 + r] = acc[g][b];
        }
    }
}

// partial[b * nrhs + r] = sum over block b's rows of A[i, r] * B[i, r]
__global__ __launch_bounds__(kRows) void dot_partial(const double* __restrict__ A, const double* __restrict__ B,
                                                     int64_t n, int nrhs, double* __restrict__ partial) {
    __shared__ double red[kRows];
    const int64_t per = (n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = int64_t(blockIdx.x) * per, hi = std::min<int64_t>(n, lo + per);
    for (int r = 0; r < nrhs; ++r) {
        double s = 0.0;
        for (int64_t i = lo + threadIdx.x; i < hi; i += kRows) s = __builtin_fma(A[i * nrhs + r], B[i * nrhs + r], s);
        red[threadIdx.x] = s;
        __syncthreads();
        for (int w = kRows / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) partial[blockIdx.x * nrhs + r] = red[0];
        __syncthreads();
    }
}

// out[r] = sum_b partial[b * nrhs + r], b ascending
__global__ void dot_final(const double* __restrict__ partial, int nblocks, int nrhs, double* __restrict__ out) {
    const int r = threadIdx.x;
    if (r >= nrhs) return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += partial[b * nrhs + r];
    out[r] = s;
}

__global__ void fill_zero(double* __restrict__ a, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) a[i] = 0.0;
}

// r = b - q
__global__ void sub_vec(const double* __restrict__ b, const double* __restrict__ q, double* __restrict__ r,
                        int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) r[i] = b[i] - q[i];
}

__global__ void copy_vec(const double* __restrict__ a, double* __restrict__ b, int64_t m) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) b[i] = a[i];
}

// alpha = rz / pq for active right-hand sides, 0 otherwise
__global__ void cg_alpha(const double* __restrict__ rz, const double* __restrict__ pq, const int* __restrict__ act,
                         int nrhs, double* __restrict__ alpha) {
    const int r = threadIdx.x;
    if (r < nrhs) alpha[r] = act[r] ? rz[r] / pq[r] : 0.0;
}

// x += alpha p, r -= alpha q
__global__ void cg_update_xr(double* __restrict__ x, double* __restrict__ res, const double* __restrict__ p,
                             const double* __restrict__ q, const double* __restrict__ alpha, int64_t n, int nrhs) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const double a = alpha[t % nrhs];
    x[t] = __builtin_fma(a, p[t], x[t]);
    res[t] = __builtin_fma(-a, q[t], res[t]);
}

// p = z + (rz_new / rz_old) p, rz_old = rz_new (active right-hand sides only)
__global__ void cg_update_p(double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ rz_new,
                            const double* __restrict__ rz_old, const int* __restrict__ act, int64_t n, int nrhs) {
    const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n * nrhs) return;
    const int r = int(t % nrhs);
    if (!act[r]) return;
    p[t] = __builtin_fma(rz_new[r] / rz_old[r], p[t], z[t]);
}

unsigned blocks_for(int64_t m, int per) { return unsigned((m + per - 1) / per); }

int twonu_of(double nu) {
    if (nu == 0.5) return 1;
    if (nu == 1.5) return 3;
    if (nu == 2.5) return 5;
    return 0;
}

template <int TWONU, int D>
hipError_t launch_matvec_d(const double* x, int64_t n, int d, double scale, const double* X, int nrhs, double* Y,
                           hipStream_t s) {
    static const ExpTable et = make_exp_table();
    for (int r0 = 0; r0 < nrhs; r0 += kMfmaRhs) {
        const int nr = std::min(kMfmaRhs, nrhs - r0);
        // column tile: a multiple of 4, at most kTileJ, with the LDS footprint within 64 KiB
        const int tj = std::min(kTileJ, ((kMfmaLds / int(sizeof(double)) - kExpSize) / (d + kMfmaRhs)) & ~3);
        const size_t lds = (kExpSize + size_t(tj) * (d + kMfmaRhs)) * sizeof(double);
        const dim3 g(blocks_for(n, kMfmaRows));
        if (nr <= 4)
            dense_matvec_mfma<TWONU, D, 1><<<g, 256, lds, s>>>(x, n, d, scale, X, nrhs, r0, nr, Y, et, tj);
        else
            dense_matvec_mfma<TWONU, D, 2><<<g, 256, lds, s>>>(x, n, d, scale, X, nrhs, r0, nr, Y, et, tj);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int TWONU>
hipError_t launch_matvec_t(const double* x, int64_t n, int d, double scale, const double* X, int nrhs, double* Y,
                           hipStream_t s) {
    switch (d) {
        case 1: return launch_matvec_d<TWONU, 1>(x, n, d, scale, X, nrhs, Y, s);
        case 2: return launch_matvec_d<TWONU, 2>(x, n, d, scale, X, nrhs, Y, s);
        case 3: return launch_matvec_d<TWONU, 3>(x, n, d, scale, X, nrhs, Y, s);
        default: return launch_matvec_d<TWONU, 0>(x, n, d, scale, X, nrhs, Y, s);
    }
}

hipError_t launch_matvec(int tn, const double* x, int64_t n, int d, double ell, const double* X, int nrhs, double* Y,
                         hipStream_t s) {
    if (tn == 1) return launch_matvec_t<1>(x, n, d, 1.0 / ell, X, nrhs, Y, s);
    if (tn == 3) return launch_matvec_t<3>(x, n, d, 1.7320508075688772 / ell, X, nrhs, Y, s);
    return launch_matvec_t<5>(x, n, d, 2.23606797749979 / ell, X, nrhs, Y, s);
}

hipError_t launch_dot(const double* A, const double* B, int64_t n, int nrhs, double* partial, double* out,
                      hipStream_t s) {
    dot_partial<<<kDotBlocks, kRows, 0, s>>>(A, B, n, nrhs, partial);
    dot_final<<<1, 64, 0, s>>>(partial, kDotBlocks, nrhs, out);
    return hipGetLastError();
}

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

struct PcgLayout {
    size_t r, z, p, q, partial, scal, act, solve, total;
};

PcgLayout pcg_layout(const kc_factor* f, int nrhs, size_t solve_bytes) {
    PcgLayout o{};
    const size_t vec = al(size_t(f->n) * nrhs * sizeof(double));
    size_t at = 0;
    o.r = at; at += vec;
    o.z = at; at += vec;
    o.p = at; at += vec;
    o.q = at; at += vec;
    o.partial = at; at += al(size_t(kDotBlocks) * nrhs * sizeof(double));
    o.scal = at; at += al(8 * size_t(nrhs) * sizeof(double));
    o.act = at; at += al(size_t(nrhs) * sizeof(int));
    o.solve = at; at += al(solve_bytes);
    o.total = at;
    return o;
}

}  // namespace

#define PCG_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t _e = (call);                                                         \
        if (_e != hipSuccess) {                                                         \
            kc::set_error(std::string(#call) + ": " + hipGetErrorString(_e));           \
            return KC_EHIP;                                                             \
        }                                                                               \
    } while (0)

extern "C" {

kc_status kc_dense_matvec(const double* x_dev, int64_t n, int32_t d, kc_kernel kernel, const double* X_dev,
                          double* Y_dev, int32_t nrhs, void* stream) {
    const int tn = twonu_of(kernel.nu);
    if (!x_dev || !X_dev || !Y_dev || n < 1 || d < 1 || d > 32 || nrhs < 1 || !tn || !(kernel.lengthscale > 0.0)) {
        kc::set_error("kc_dense_matvec: need points, n >= 1, 1 <= d <= 32, nrhs >= 1, nu in {0.5,1.5,2.5}, l > 0");
        return KC_EINVAL;
    }
    if (X_dev == Y_dev) {
        kc::set_error("kc_dense_matvec: X and Y must not alias");
        return KC_EINVAL;
    }
    PCG_HIP(launch_matvec(tn, x_dev, n, d, kernel.lengthscale, X_dev, nrhs, Y_dev, static_cast<hipStream_t>(stream)));
    return KC_OK;
}

kc_status kc_pcg_bytes(const kc_factor* f, int32_t nrhs, size_t* bytes) {
    if (!f || !bytes || nrhs < 1) return KC_EINVAL;
    size_t sb = 0;
    kc_status st = kc_solve_bytes(f, nrhs, &sb);
    if (st != KC_OK) return st;
    *bytes = pcg_layout(f, nrhs, sb).total;
    return KC_OK;
}

kc_status kc_pcg(kc_factor* f, const double* x_dev, kc_kernel kernel, const double* b_dev, double* sol_dev,
                 int32_t nrhs, double tol, int32_t maxit, void* scratch_dev, size_t scratch_bytes, void* stream,
                 kc_pcg_info_t* info) {
    const int tn = twonu_of(kernel.nu);
    if (!f || !x_dev || !b_dev || !sol_dev || !scratch_dev || !info || nrhs < 1 || !tn ||
        !(kernel.lengthscale > 0.0) || !(tol > 0.0) || maxit < 1 || f->d > 32) {
        kc::set_error("kc_pcg: invalid argument");
        return KC_EINVAL;
    }
    if (!f->factorized) {
        kc::set_error("kc_pcg: factor has not been computed");
        return KC_ESTATE;
    }
    size_t sb = 0;
    kc_status st = kc_solve_bytes(f, nrhs, &sb);
    if (st != KC_OK) return st;
    const PcgLayout o = pcg_layout(f, nrhs, sb);
    if (scratch_bytes < o.total || reinterpret_cast<uintptr_t>(scratch_dev) % 256) {
        kc::set_error("kc_pcg: scratch must be 256-byte aligned and hold kc_pcg_bytes bytes");
        return KC_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(scratch_dev);
    double* r = reinterpret_cast<double*>(base + o.r);
    double* z = reinterpret_cast<double*>(base + o.z);
    double* p = reinterpret_cast<double*>(base + o.p);
    double* q = reinterpret_cast<double*>(base + o.q);
    double* partial = reinterpret_cast<double*>(base + o.partial);
    double* sc = reinterpret_cast<double*>(base + o.scal);
    double* rz = sc;                  // [nrhs]
    double* rz_new = sc + nrhs;       // [nrhs]
    double* pq = sc + 2 * nrhs;       // [nrhs]
    double* alpha = sc + 3 * nrhs;    // [nrhs]
    double* rr = sc + 4 * nrhs;       // [nrhs]
    double* bb = sc + 5 * nrhs;       // [nrhs]
    int* act = reinterpret_cast<int*>(base + o.act);
    void* solve_scratch = base + o.solve;
    const int64_t m = f->n * int64_t(nrhs);
    const unsigned gb = blocks_for(m, 256);

    hipEvent_t e0 = nullptr, e1 = nullptr;
    struct EventGuard {
        hipEvent_t* a;
        hipEvent_t* b;
        ~EventGuard() {
            if (*a) (void)hipEventDestroy(*a);
            if (*b) (void)hipEventDestroy(*b);
        }
    } guard{&e0, &e1};
    PCG_HIP(hipEventCreate(&e0));
    PCG_HIP(hipEventCreate(&e1));
    float t_mv = 0.f, t_pc = 0.f, ms = 0.f;

    std::vector<double> hb(nrhs), hr(nrhs);
    std::vector<int> hact(nrhs, 1);
    fill_zero<<<gb, 256, 0, s>>>(sol_dev, m);
    copy_vec<<<gb, 256, 0, s>>>(b_dev, r, m);
    PCG_HIP(launch_dot(b_dev, b_dev, f->n, nrhs, partial, bb, s));
    PCG_HIP(hipMemcpyAsync(hb.data(), bb, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
    PCG_HIP(hipMemcpyAsync(act, hact.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
    PCG_HIP(hipEventRecord(e0, s));
    st = kc_solve(f, r, z, nrhs, solve_scratch, sb, stream);
    if (st != KC_OK) return st;
    PCG_HIP(hipEventRecord(e1, s));
    PCG_HIP(hipStreamSynchronize(s));
    PCG_HIP(hipEventElapsedTime(&ms, e0, e1));
    t_pc += ms;
    copy_vec<<<gb, 256, 0, s>>>(z, p, m);
    PCG_HIP(launch_dot(r, z, f->n, nrhs, partial, rz, s));

    // True residual r = b - Theta x (one dense product), which replaces the
    // recursively updated one; returns max over right-hand sides of ||r||/||b||
    // and marks the right-hand sides still above tol as active.
    std::vector<double> hrel(nrhs, 0.0);
    auto true_residual = [&](double& out) -> hipError_t {
        hipError_t e;
        if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
        if ((e = launch_matvec(tn, x_dev, f->n, f->d, kernel.lengthscale, sol_dev, nrhs, q, s)) != hipSuccess) return e;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
        sub_vec<<<gb, 256, 0, s>>>(b_dev, q, r, m);
        if ((e = launch_dot(r, r, f->n, nrhs, partial, rr, s)) != hipSuccess) return e;
        if ((e = hipMemcpyAsync(hr.data(), rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, s)) != hipSuccess)
            return e;
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return e;
        if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) return e;
        t_mv += ms;
        out = 0.0;
        for (int k = 0; k < nrhs; ++k) {
            hrel[k] = hb[k] > 0.0 ? std::sqrt(hr[k] / hb[k]) : 0.0;
            out = std::max(out, hrel[k]);
            hact[k] = hrel[k] > tol ? 1 : 0;
        }
        return hipSuccess;
    };

    int it = 0, restarts = 0;
    double worst = 0.0, true_worst = -1.0;
    bool done = false;
    for (it = 1; it <= maxit; ++it) {
        PCG_HIP(hipEventRecord(e0, s));
        PCG_HIP(launch_matvec(tn, x_dev, f->n, f->d, kernel.lengthscale, p, nrhs, q, s));
        PCG_HIP(hipEventRecord(e1, s));
        PCG_HIP(launch_dot(p, q, f->n, nrhs, partial, pq, s));
        cg_alpha<<<1, 64, 0, s>>>(rz, pq, act, nrhs, alpha);
        cg_update_xr<<<gb, 256, 0, s>>>(sol_dev, r, p, q, alpha, f->n, nrhs);
        PCG_HIP(launch_dot(r, r, f->n, nrhs, partial, rr, s));
        PCG_HIP(hipMemcpyAsync(hr.data(), rr, nrhs * sizeof(double), hipMemcpyDeviceToHost, s));
        PCG_HIP(hipStreamSynchronize(s));
        PCG_HIP(hipEventElapsedTime(&ms, e0, e1));
        t_mv += ms;
        worst = 0.0;
        bool any = false;
        for (int k = 0; k < nrhs; ++k) {
            const double rel = hb[k] > 0.0 ? std::sqrt(hr[k] / hb[k]) : 0.0;
            worst = std::max(worst, rel);
            if (hact[k] && rel <= tol) hact[k] = 0;
            any = any || hact[k];
        }
        if (!any) {
            // the recursive residual has converged: confirm with the true one, and
            // where rounding let the two drift apart, restart CG from the current x
            PCG_HIP(true_residual(true_worst));
            if (true_worst <= tol || it == maxit) {
                done = true_worst <= tol;
                break;
            }
            ++restarts;
            PCG_HIP(hipMemcpyAsync(act, hact.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
            PCG_HIP(hipEventRecord(e0, s));
            st = kc_solve(f, r, z, nrhs, solve_scratch, sb, stream);
            if (st != KC_OK) return st;
            PCG_HIP(hipEventRecord(e1, s));
            copy_vec<<<gb, 256, 0, s>>>(z, p, m);
            PCG_HIP(launch_dot(r, z, f->n, nrhs, partial, rz, s));
            PCG_HIP(hipStreamSynchronize(s));
            PCG_HIP(hipEventElapsedTime(&ms, e0, e1));
            t_pc += ms;
            true_worst = -1.0;
            continue;
        }
        PCG_HIP(hipMemcpyAsync(act, hact.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        PCG_HIP(hipEventRecord(e0, s));
        st = kc_solve(f, r, z, nrhs, solve_scratch, sb, stream);
        if (st != KC_OK) return st;
        PCG_HIP(hipEventRecord(e1, s));
        PCG_HIP(launch_dot(r, z, f->n, nrhs, partial, rz_new, s));
        cg_update_p<<<gb, 256, 0, s>>>(p, z, rz_new, rz, act, f->n, nrhs);
        copy_vec<<<1, 64, 0, s>>>(rz_new, rz, nrhs);
        PCG_HIP(hipStreamSynchronize(s));
        PCG_HIP(hipEventElapsedTime(&ms, e0, e1));
        t_pc += ms;
    }
    PCG_HIP(hipStreamSynchronize(s));
    if (true_worst < 0.0) PCG_HIP(true_residual(true_worst));  // stopped at maxit
    info->iterations = std::min(it, maxit);
    info->converged = done ? 1 : 0;
    info->max_rel_residual = worst;
    info->true_rel_residual = true_worst;
    info->restarts = restarts;
    info->t_matvec_ms = t_mv;
    info->t_precond_ms = t_pc;
    return KC_OK;
}

}  // extern "C"
