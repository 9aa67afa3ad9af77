// Dense covariance matvec and preconditioned conjugate gradients (gfx950).
//
// The sparse factor is used as a preconditioner for CG on the dense system
// Theta x = b (Section 4.3 suggests CG with the factor when the approximation
// alone is not accurate enough).  Each iteration needs one product with the
// dense N x N Theta, whose entries are generated on the fly: the work is N^2
// evaluations of the kernel (a square root and an exponential each), bound by
// the FP64 vector ALUs, not by memory and not by matrix cores -- there is no
// reusable operand to contract.  Rows are owned by threads; columns stream
// through LDS in tiles shared by the 256 rows of a block.
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
constexpr int kTileJ = 256;      // columns staged per LDS tile
constexpr int kDotBlocks = 512;  // fixed grid of the dot-product reduction
constexpr int kMaxNr = 8;

template <int TWONU>
__device__ __forceinline__ double matern_fast(double r, double inv_ell) {
    if constexpr (TWONU == 1) {
        return exp(-r * inv_ell);
    } else if constexpr (TWONU == 3) {
        const double a = 1.7320508075688772 * r * inv_ell;
        return (1.0 + a) * exp(-a);
    } else {
        const double a = 2.23606797749979 * r * inv_ell;
        return (1.0 + a + a * a * (1.0 / 3.0)) * exp(-a);
    }
}

// Y[i, r0+r] = sum_j Theta(x_i, x_j) X[j, r0+r], j ascending.  x: n x d (any order,
// X and Y in the same order).  D = d for d <= 3 (coordinates in registers), D = 0
// for any d <= 32 (own coordinates re-read through the cache).
template <int TWONU, int NR, int D>
__global__ __launch_bounds__(kRows) void dense_matvec(const double* __restrict__ x, int64_t n, int d, double inv_ell,
                                                      const double* __restrict__ X, int ld, int r0,
                                                      double* __restrict__ Y) {
    extern __shared__ double tile[];  // kTileJ * d coordinates, then kTileJ * NR values
    double* sx = tile;
    double* sv = tile + size_t(kTileJ) * d;
    const int64_t i = int64_t(blockIdx.x) * kRows + threadIdx.x;
    const int64_t ic = i < n ? i : n - 1;
    double xi[D > 0 ? D : 1];
#pragma unroll
    for (int t = 0; t < (D > 0 ? D : 1); ++t) xi[t] = D > 0 ? x[ic * D + t] : 0.0;
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    for (int64_t j0 = 0; j0 < n; j0 += kTileJ) {
        const int m = int(n - j0 < kTileJ ? n - j0 : kTileJ);
        for (int q = threadIdx.x; q < m * d; q += kRows) sx[q] = x[j0 * d + q];
        for (int q = threadIdx.x; q < m * NR; q += kRows) sv[q] = X[(j0 + q / NR) * ld + r0 + q % NR];
        __syncthreads();
        for (int jj = 0; jj < m; ++jj) {
            double s = 0.0;
            if constexpr (D > 0) {
#pragma unroll
                for (int t = 0; t < D; ++t) {
                    const double df = xi[t] - sx[jj * D + t];
                    s = __builtin_fma(df, df, s);
                }
            } else {
                for (int t = 0; t < d; ++t) {
                    const double df = x[ic * d + t] - sx[jj * d + t];
                    s = __builtin_fma(df, df, s);
                }
            }
            const double th = matern_fast<TWONU>(__builtin_sqrt(s), inv_ell);
#pragma unroll
            for (int r = 0; r < NR; ++r) acc[r] = __builtin_fma(th, sv[jj * NR + r], acc[r]);
        }
        __syncthreads();
    }
    if (i < n) {
#pragma unroll
        for (int r = 0; r < NR; ++r) Y[i * ld + r0 + r] = acc[r];
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
hipError_t launch_matvec_d(const double* x, int64_t n, int d, double inv_ell, const double* X, int nrhs, double* Y,
                           hipStream_t s) {
    for (int r0 = 0; r0 < nrhs; r0 += kMaxNr) {
        const int nr = std::min(kMaxNr, nrhs - r0);
        const size_t lds = size_t(kTileJ) * (d + nr) * sizeof(double);
        const dim3 g(blocks_for(n, kRows));
        switch (nr) {
            case 1: dense_matvec<TWONU, 1, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 2: dense_matvec<TWONU, 2, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 3: dense_matvec<TWONU, 3, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 4: dense_matvec<TWONU, 4, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 5: dense_matvec<TWONU, 5, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 6: dense_matvec<TWONU, 6, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            case 7: dense_matvec<TWONU, 7, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
            default: dense_matvec<TWONU, 8, D><<<g, kRows, lds, s>>>(x, n, d, inv_ell, X, nrhs, r0, Y); break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <int TWONU>
hipError_t launch_matvec_t(const double* x, int64_t n, int d, double inv_ell, const double* X, int nrhs, double* Y,
                           hipStream_t s) {
    switch (d) {
        case 1: return launch_matvec_d<TWONU, 1>(x, n, d, inv_ell, X, nrhs, Y, s);
        case 2: return launch_matvec_d<TWONU, 2>(x, n, d, inv_ell, X, nrhs, Y, s);
        case 3: return launch_matvec_d<TWONU, 3>(x, n, d, inv_ell, X, nrhs, Y, s);
        default: return launch_matvec_d<TWONU, 0>(x, n, d, inv_ell, X, nrhs, Y, s);
    }
}

hipError_t launch_matvec(int tn, const double* x, int64_t n, int d, double ell, const double* X, int nrhs, double* Y,
                         hipStream_t s) {
    const double inv = 1.0 / ell;
    if (tn == 1) return launch_matvec_t<1>(x, n, d, inv, X, nrhs, Y, s);
    if (tn == 3) return launch_matvec_t<3>(x, n, d, inv, X, nrhs, Y, s);
    return launch_matvec_t<5>(x, n, d, inv, X, nrhs, Y, s);
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

    int it = 0;
    double worst = 0.0;
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
            done = true;
            break;
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
    info->iterations = done ? it : maxit;
    info->converged = done ? 1 : 0;
    info->max_rel_residual = worst;
    info->t_matvec_ms = t_mv;
    info->t_precond_ms = t_pc;
    return KC_OK;
}

}  // extern "C"
