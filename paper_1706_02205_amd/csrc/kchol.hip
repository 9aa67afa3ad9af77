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
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <climits>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <atomic>
#include <thread>
#include <string>
#include <system_error>
#include <type_traits>
#include <vector>

#include "crmath.h"
#include "factor.h"
#include "plan.h"

using kc::Unit;

namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;                    // 4 wavefronts
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int64_t kLongColumn = 2048;          // backward solve: longer columns are reduced in pieces
constexpr int64_t kChunk = 512;                // entries per partial dot product of a long top part
constexpr int64_t kFinePiece = 2048;           // entries per piece of a top column's rows below the top block
constexpr int64_t kBandRows = 32768;           // rows per band of those pieces (8 RHS: 2 MB of x per band)
constexpr int kMaxRhsPerPass = 8;

enum Counter {
    kNonpos = 0, kShifted = 1, kUpdates = 2, kExpHard = 3, kNonfinite = 4, kMatchErr = 5, kMatchTotal = 6,
    kNumCounters = 8
};

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

// The longest walk of each 64-entry work unit: over the unit's entries (k,j),
// the prefix of row k that precedes (k,j).  One wavefront per unit.
__global__ __launch_bounds__(kBlock) void unit_walk_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                           const int64_t* __restrict__ colptr,
                                                           const int32_t* __restrict__ rowidx,
                                                           const uint32_t* __restrict__ csc2csr,
                                                           const int64_t* __restrict__ rowptr,
                                                           int32_t* __restrict__ walk) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= nunits) return;
    const int lane = threadIdx.x % kWave;
    const int j = units[u].col;
    const int64_t e = colptr[j] + units[u].first + lane;
    long long w = 0;
    if (e < colptr[j + 1]) w = (long long)csc2csr[e] - (long long)rowptr[rowidx[e]];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const long long o = __shfl_xor(w, off, kWave);
        w = o > w ? o : w;
    }
    if (lane == 0) walk[u] = int32_t(w < INT32_MAX ? w : INT32_MAX);
}

// ---------------------------------------------------------------------------
// Wave-local LDS ordering: every lane's LDS writes are visible to the other
// lanes of the same wavefront after this point.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Row windows.  L2 lines are 128 bytes, and with thousands of rows walked at
// once a line is evicted before a lane comes back for its other half, so every
// load below reads whole lines: 64 column-index gaps (16 bits each, 128 B) per
// window, and their values in 16-entry pieces (128 B each, FP64) or 32-entry
// pieces (128 B, FP32).  Rows start on 64-entry boundaries, so windows are
// line-aligned.
constexpr int kWin = 64;
constexpr int kEscQ = 2;  // escapes of a row held in registers; later ones are read when met
static_assert(kWin == kc::kRowAlign, "row windows must match the row alignment of the plan");

__device__ __forceinline__ void load_gaps(const uint32_t* __restrict__ cdelta, int64_t p, uint32_t (&w)[kWin / 2]) {
    const uint4* ip = reinterpret_cast<const uint4*>(cdelta + p / 2);
#pragma unroll
    for (int q = 0; q < kWin / 8; ++q) {
        const uint4 v = ip[q];
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
    }
}

template <int N>
__device__ __forceinline__ void load_vals(const double* __restrict__ Lv, int64_t p, double (&val)[N]) {
    const double2* vp = reinterpret_cast<const double2*>(Lv + p);
#pragma unroll
    for (int q = 0; q < N / 2; ++q) {
        const double2 v = vp[q];
        val[2 * q] = v.x;
        val[2 * q + 1] = v.y;
    }
}

template <int N>
__device__ __forceinline__ void load_vals(const float* __restrict__ Lv, int64_t p, float (&val)[N]) {
    const float4* vp = reinterpret_cast<const float4*>(Lv + p);
#pragma unroll
    for (int q = 0; q < N / 4; ++q) {
        const float4 v = vp[q];
        val[4 * q] = v.x;
        val[4 * q + 1] = v.y;
        val[4 * q + 2] = v.z;
        val[4 * q + 3] = v.w;
    }
}

// Workgroups are dealt to the 8 XCDs round-robin (block b runs on XCD b % 8).
// Renumber them so that each XCD receives one contiguous range of blocks: the
// rows and columns of a solve level are laid out in spatial order, so each
// XCD's L2 then serves one region of the point cloud.  (The factorization's
// units are ordered by length instead, and keep the plain block order.)
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int q = nb / kNumXcd, r = nb % kNumXcd;
    const int x = b % kNumXcd, i = b / kNumXcd;
    return x * q + (x < r ? x : r) + i;
}

// ---------------------------------------------------------------------------
// A1+A2: Theta on S fused into ICHOL(0), one DAG level per launch.
//
// Left-looking form of the paper's incomplete Cholesky: entry (k,j) of column j
// starts at Theta_kj and receives, for every parent i < j with (j,i) and (k,i)
// in S, in ascending i, the update A_kj <- fma(-L_ki, L_ji, A_kj) -- the same
// operations in the same order as the right-looking algorithm of Section 2.2,
// so the FP64 result is bitwise that algorithm's.  All parents of column j lie
// in earlier levels, so the columns of one level are independent.
//
// A wavefront owns 64 consecutive entries of one column (a Unit), one entry k
// per lane.  Row j's parents (indices and L_ji) are staged once in LDS.  Each
// lane then streams row k of L -- stored by rows, padded to 32-entry windows --
// from its start up to the entry (k,j), whose position is known from the
// CSC->CSR map, and merges it against the staged row j with a cursor.  The pivot
// A_jj is accumulated by every wave of column j from the staged row j, so the
// chunks of a long column need no communication.
//
// VT = double: FP64.  VT = float (MIXED): off-diagonal Theta, updates and the
// stored L in FP32; the pivot accumulates exact FP32 x FP32 products in FP64,
// and sqrt and the division by L_jj are FP64.
// Everything one work unit reads and writes.
template <typename VT>
struct IcholArgs {
    const int64_t* colptr;
    const int32_t* rowidx;
    const uint32_t* csc2csr;
    const int64_t* rowptr;
    const int64_t* rowend;
    const int32_t* colidx;
    const uint32_t* cdelta;
    const uint32_t* escptr;
    const int32_t* esc;
    VT* Lv;
    VT* Lcsc;
    double* diag;
    const double* xh;
    int d;
    double ell;
    const int32_t* inst;
    const double* ells;
    int policy;
    double tau;
    int cap;
    int stage_max;  // rows with more parents are read from device memory, not staged
    int nbuck;  // 0: cursor merge; else buckets of the staged row's directory (a power of 2)
    unsigned long long* counters;
    // match masks (see match_masks_kernel), or null: per CSC entry a word offset and
    // walk end (mmeta), and the mask words (mwords, mwords_n of them)
    const uint64_t* mmeta;
    const uint64_t* mwords;
    uint64_t mwords_n;
};

// Match masks.  For an entry (k,j) below the diagonal the factorization needs
// the parents i < j common to row k and row j, in ascending order.  Two bit
// masks record them once per pattern: mk over row k's entries before (k,j)
// (bit t: the row's t-th entry is a parent of j) and mj over row j's parents
// (bit s: the s-th parent of j is in row k).  The t-th set bit of mk and the
// t-th set bit of mj name the same i.  The entry's meta word holds the offset
// of mk (mj follows, ceil(pos/64) words later) and, above bit kMatchOffBits,
// one past the last set bit of mk (the walk ends there).
constexpr int kMatchOffBits = 40;
constexpr uint64_t kMatchOffMask = (uint64_t(1) << kMatchOffBits) - 1;

// ---------------------------------------------------------------------------
// Match masks (see factor_entries_mask), built once per pattern.
//
// Words of an entry e = (k,j) below the diagonal: ceil(pos/64) for mk (pos =
// entries of row k before (k,j)) plus ceil(np/64) for mj (np = parents of j);
// none for the diagonal.  Offsets are an exclusive prefix sum of the word
// counts over the plan's units (each CSC entry lies in exactly one unit): a
// block of four units scans its 256 entries in LDS (match_count_kernel), the
// host scans the block totals, and match_base_kernel adds them.

__device__ __forceinline__ uint64_t match_words_of(const int64_t* __restrict__ colptr,
                                                   const int32_t* __restrict__ rowidx,
                                                   const uint32_t* __restrict__ csc2csr,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int64_t* __restrict__ rowend, int j, int64_t e) {
    const int k = rowidx[e];
    if (k == j) return 0;
    const int64_t pos = int64_t(csc2csr[e]) - rowptr[k];
    const int64_t np = rowend[j] - 1 - rowptr[j];
    return uint64_t((pos + 63) >> 6) + uint64_t((np + 63) >> 6);
}

// Sum of the words over all entries into counters[kMatchTotal] (grid-stride over
// units, one atomic per workgroup).
__global__ __launch_bounds__(kBlock) void match_total_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                             const int64_t* __restrict__ colptr,
                                                             const int32_t* __restrict__ rowidx,
                                                             const uint32_t* __restrict__ csc2csr,
                                                             const int64_t* __restrict__ rowptr,
                                                             const int64_t* __restrict__ rowend,
                                                             unsigned long long* __restrict__ counters) {
    __shared__ unsigned long long part[kWavesPerBlock];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    unsigned long long acc = 0;
    for (int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave; u < nunits;
         u += int64_t(gridDim.x) * kWavesPerBlock) {
        const int j = units[u].col;
        const int64_t e = colptr[j] + units[u].first + lane;
        if (e < colptr[j + 1]) acc += match_words_of(colptr, rowidx, csc2csr, rowptr, rowend, j, e);
    }
    acc = wave_sum(acc);
    if (lane == 0) part[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kWavesPerBlock; ++w) t += part[w];
        if (t) atomicAdd(counters + kMatchTotal, t);
    }
}

// meta[e] = exclusive prefix of the words within the block; bsum[block] = block total.
__global__ __launch_bounds__(kBlock) void match_count_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                             const int64_t* __restrict__ colptr,
                                                             const int32_t* __restrict__ rowidx,
                                                             const uint32_t* __restrict__ csc2csr,
                                                             const int64_t* __restrict__ rowptr,
                                                             const int64_t* __restrict__ rowend,
                                                             uint64_t* __restrict__ meta, uint64_t* __restrict__ bsum) {
    __shared__ uint64_t sc[kBlock];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave;
    int64_t e = -1;
    uint64_t w = 0;
    if (u < nunits) {
        const int j = units[u].col;
        e = colptr[j] + units[u].first + lane;
        if (e < colptr[j + 1]) w = match_words_of(colptr, rowidx, csc2csr, rowptr, rowend, j, e);
        else e = -1;
    }
    sc[threadIdx.x] = w;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {  // inclusive scan (Hillis-Steele)
        const uint64_t add = threadIdx.x >= unsigned(off) ? sc[threadIdx.x - off] : 0;
        __syncthreads();
        sc[threadIdx.x] += add;
        __syncthreads();
    }
    if (e >= 0) meta[e] = sc[threadIdx.x] - w;
    if (threadIdx.x == kBlock - 1) bsum[blockIdx.x] = sc[threadIdx.x];
}

// meta[e] += base[block] (base: exclusive prefix of the block totals)
__global__ __launch_bounds__(kBlock) void match_base_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                            const int64_t* __restrict__ colptr,
                                                            const uint64_t* __restrict__ base,
                                                            uint64_t* __restrict__ meta) {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= nunits) return;
    const int j = units[u].col;
    const int64_t e = colptr[j] + units[u].first + lane;
    if (e < colptr[j + 1]) meta[e] += base[blockIdx.x];
}

__global__ void fill_u64(uint64_t* __restrict__ p, uint64_t m, uint64_t v) {
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < m; i += stride) p[i] = v;
}

// The masks of one unit per wave: row j's parents staged in the wave's LDS, each
// lane walks row k's indices before (k,j) with a cursor over them and sets a bit
// of mk for each of its entries found in row j and the bit of mj of the parent
// it found.  mj words a lane never reaches stay as zeroed beforehand; meta[e]
// gets the walk end (one past the last match) above its offset.
__global__ __launch_bounds__(kBlock) void match_masks_kernel(const Unit* __restrict__ units, int64_t nunits,
                                                             const int64_t* __restrict__ colptr,
                                                             const int32_t* __restrict__ rowidx,
                                                             const uint32_t* __restrict__ csc2csr,
                                                             const int64_t* __restrict__ rowptr,
                                                             const int64_t* __restrict__ rowend,
                                                             const int32_t* __restrict__ colidx, int cap,
                                                             uint64_t* __restrict__ meta, uint64_t* __restrict__ words,
                                                             uint64_t nwords, unsigned long long* __restrict__ counters) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t u = int64_t(blockIdx.x) * kWavesPerBlock + wave;
    if (u >= nunits) return;  // whole wave; only wave-level LDS ordering below
    int32_t* sidx = reinterpret_cast<int32_t*>(smem) + int64_t(wave) * cap;
    const int j = __builtin_amdgcn_readfirstlane(units[u].col);
    const int first = __builtin_amdgcn_readfirstlane(units[u].first);
    const int64_t t0 = rowptr[j];
    const int np = int(rowend[j] - 1 - t0);
    for (int t = lane; t < np; t += kWave) sidx[t] = colidx[t0 + t];
    if (lane == 0) sidx[np] = INT_MAX;
    wave_lds_sync();
    const int64_t e = colptr[j] + first + lane;
    if (e >= colptr[j + 1]) return;
    const int k = rowidx[e];
    const uint64_t base = meta[e] & kMatchOffMask;
    if (k == j) return;  // no walk: offset only
    const int64_t rp = rowptr[k];
    const int pos = int(int64_t(csc2csr[e]) - rp);
    const int nk = (pos + 63) >> 6, nj = (np + 63) >> 6;
    if (base + uint64_t(nk) + uint64_t(nj) > nwords) {
        atomicAdd(counters + kMatchErr, 1ull);
        return;
    }
    uint64_t* __restrict__ mk = words + base;
    uint64_t* __restrict__ mj = mk + nk;
    int q = 0, jcur = 0, last = -1;
    uint64_t kw = 0, jwv = 0;
    for (int t0w = 0; t0w < pos; t0w += 4) {
        const int4 iv = *reinterpret_cast<const int4*>(colidx + rp + t0w);  // rows start 64-aligned
        const int ci[4] = {iv.x, iv.y, iv.z, iv.w};
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            const int t = t0w + h;
            if (t < pos) {
                const int i = ci[h];
                while (sidx[q] < i) ++q;  // the sentinel stops the cursor at np
                if (sidx[q] == i) {
                    kw |= uint64_t(1) << (t & 63);
                    last = t;
                    const int qw = q >> 6;
                    if (qw != jcur) {
                        mj[jcur] = jwv;
                        jcur = qw;
                        jwv = 0;
                    }
                    jwv |= uint64_t(1) << (q & 63);
                }
                if ((t & 63) == 63) {
                    mk[t >> 6] = kw;
                    kw = 0;
                }
            }
        }
    }
    if (pos & 63) mk[pos >> 6] = kw;
    if (nj > 0) mj[jcur] = jwv;
    meta[e] = base | (uint64_t(last + 1) << kMatchOffBits);
}

// Row j's parents (indices and L_ji) into the workgroup's LDS, staged by all its
// threads once for every wave of the block; returns their number.
template <typename VT>
__device__ __forceinline__ int stage_row(const IcholArgs<VT>& a, int j, VT* sval, int32_t* sidx) {
    const int64_t t0 = a.rowptr[j];
    const int np = int(a.rowend[j] - 1 - t0);  // row j without its diagonal
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
        sidx[t] = a.colidx[t0 + t];
        sval[t] = a.Lv[t0 + t];
    }
    if (threadIdx.x == 0) sidx[np] = INT_MAX;  // sentinel ends every cursor walk
    return np;
}

// Bucket directory of the staged row for long rows: bucket b holds the parents i
// with i >> shift == b, at positions [sb[b], sb[b+1]) of sidx (nb buckets cover
// [0, j)).  A lookup is then one directory read and a probe or two, independent
// of the other lookups, instead of a cursor that advances one dependent LDS read
// at a time.  Built by all threads of the workgroup; returns the shift.
__device__ __forceinline__ int build_buckets(const int32_t* sidx, int np, int j, int nb, uint16_t* sb) {
    int shift = 0;
    while ((j >> shift) >= nb) ++shift;
    for (int q = threadIdx.x; q < np; q += blockDim.x) {
        const int bq = sidx[q] >> shift, bp = q ? (sidx[q - 1] >> shift) : -1;
        for (int b = bp + 1; b <= bq; ++b) sb[b] = uint16_t(q);
    }
    const int bl = np ? (sidx[np - 1] >> shift) : -1;
    for (int b = bl + 1 + int(threadIdx.x); b <= nb; b += int(blockDim.x)) sb[b] = uint16_t(np);
    return shift;
}

// 64 consecutive entries of column j starting at `first` (first < length of the
// column), one per lane of the wave; sval/sidx hold row j's np parents (and sb,
// when BUCKETS, their directory with the given shift).
template <int TWONU, bool COUNT, typename VT, bool BUCKETS>
__device__ __forceinline__ void factor_entries(const IcholArgs<VT>& a, int j, int first, int np, int lane,
                                               const VT* sval, const int32_t* sidx, const uint16_t* sb,
                                               int shift) {
    const int64_t* __restrict__ colptr = a.colptr;
    const int32_t* __restrict__ rowidx = a.rowidx;
    const uint32_t* __restrict__ csc2csr = a.csc2csr;
    const int64_t* __restrict__ rowptr = a.rowptr;
    const uint32_t* __restrict__ cdelta = a.cdelta;
    const uint32_t* __restrict__ escptr = a.escptr;
    const int32_t* __restrict__ esc = a.esc;
    VT* __restrict__ Lv = a.Lv;
    VT* __restrict__ Lcsc = a.Lcsc;
    double* __restrict__ diag = a.diag;
    const double* __restrict__ xh = a.xh;
    const int d = a.d, policy = a.policy;
    const double tau = a.tau;
    double ell = a.ell;
    unsigned long long* __restrict__ counters = a.counters;

    double dacc = 1.0;  // Theta_jj
    for (int t = 0; t < np; ++t) {
        double v = double(sval[t]);
        dacc = __builtin_fma(-v, v, dacc);
    }

    const int64_t e = colptr[j] + first + lane;
    const bool active = e < colptr[j + 1];
    const int k = active ? rowidx[e] : j;
    if (a.ells) ell = a.ells[a.inst[j]];  // a batch: lengthscale of j's instance
    int hard = 0;
    VT acc;
    if constexpr (sizeof(VT) == 8)
        acc = kcdev::matern<TWONU>(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d), ell, hard);
    else
        acc = kcdev::matern_f32<TWONU>(float(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d)), float(ell));

    unsigned long long hits = 0;
    if (active) {
        const int64_t pend = csc2csr[e];  // position of (k,j) in row k
        int q = 0;
        // the row's column indices, decoded from the 16-bit gaps: a zero gap is an
        // escape whose index comes from the row's escape list (first kEscQ in registers)
        const uint32_t eb = escptr[k], ee = escptr[k + 1];
        // a queue in named registers (an array would be indexed at run time, in scratch)
        int e0 = eb < ee ? esc[eb] : 0, e1 = eb + 1 < ee ? esc[eb + 1] : 0;
        static_assert(kEscQ == 2, "the escape queue below holds 2 entries");
        uint32_t ec = 0;  // escapes met so far
        int cur = -1;     // index of the last decoded entry
        // values of one load: FP64 in 16-entry pieces, FP32 32-entry pieces (one line each).
        // Loading more FP64 values at once costs registers, hence occupancy, and
        // measured slower; so did 8-entry pieces (more round trips).
        constexpr int kPiece = sizeof(VT) == 8 ? 16 : 32;
        for (int64_t p = rowptr[k]; p < pend; p += kWin) {
            const int lim = pend - p < kWin ? int(pend - p) : kWin;  // entries of this window before (k,j)
            uint32_t gw[kWin / 2];
            load_gaps(cdelta, p, gw);
#pragma unroll
            for (int off = 0; off < kWin; off += kPiece) {
                if (off < lim) {
                    VT val[kPiece];
                    load_vals(Lv, p + off, val);
#pragma unroll
                    for (int t = 0; t < kPiece; ++t) {
                        if (off + t < lim) {
                            const uint32_t g = (gw[(off + t) >> 1] >> (((off + t) & 1) * 16)) & 0xffffu;
                            if (g) {
                                cur += int(g);
                            } else {
                                cur = ec < kEscQ ? e0 : esc[eb + ec];
                                e0 = e1;
                                ++ec;
                            }
                            const int i = cur;
                            int hit;
                            if constexpr (BUCKETS) {
                                const int b = i >> shift;
                                const int q0 = sb[b], qe = sb[b + 1];
                                const int c0 = sidx[q0], c1 = sidx[q0 + 1];  // q0 + 1 <= np + 1 < cap
                                hit = (q0 < qe && c0 == i) ? q0 : (q0 + 1 < qe && c1 == i) ? q0 + 1 : -1;
                                if (hit < 0 && qe - q0 > 2) {  // a crowded bucket: scan the rest
                                    for (int r = q0 + 2; r < qe; ++r)
                                        if (sidx[r] == i) {
                                            hit = r;
                                            break;
                                        }
                                }
                            } else {
                                while (sidx[q] < i) ++q;
                                hit = sidx[q] == i ? q : -1;
                            }
                            if (hit >= 0) {
                                const VT lji = sval[hit];
                                if constexpr (sizeof(VT) == 8) acc = __builtin_fma(-val[t], lji, acc);
                                else acc = __builtin_fmaf(-val[t], lji, acc);
                                if (COUNT && lji != VT(0)) ++hits;
                            }
                        }
                    }
                }
            }
        }
    }

    bool zero = false, shifted = false;
    double piv = dacc;
    if (policy == KC_PIVOT_ZERO) {
        zero = !(piv > 0.0);
    } else {
        const double fl = tau * 1.0;
        if (!(piv > fl)) {
            piv = fl;
            shifted = true;
        }
    }
    const double ljj = zero ? 0.0 : __builtin_sqrt(piv);
    bool bad = false;
    if (active) {
        VT out;
        if (zero) out = VT(0);
        else if (k == j) out = VT(ljj);
        else if constexpr (sizeof(VT) == 8) out = acc / ljj;
        else out = float(double(acc) / ljj);
        Lv[csc2csr[e]] = out;
        Lcsc[e] = out;
        if constexpr (sizeof(VT) == 4)
            if (k == j) diag[j] = ljj;
        bad = !__builtin_isfinite(out);
    }
    // entries of L that came out inf or NaN (e.g. after a tiny shifted pivot): one atomic per wave
    const unsigned long long nf = __ballot(bad);
    if (nf && lane == 0) atomicAdd(counters + kNonfinite, (unsigned long long)__popcll(nf));
    if (first == 0 && lane == 0) {
        if (zero) atomicAdd(counters + kNonpos, 1ull);
        if (shifted) atomicAdd(counters + kShifted, 1ull);
    }
    if (COUNT) {
        const unsigned long long tot = wave_sum(hits);
        if (lane == 0 && tot) atomicAdd(counters + kUpdates, tot);
    }
    if (hard && active) atomicAdd(counters + kExpHard, 1ull);
}

// Row j's parent values alone (the masked factorization needs no indices).
template <typename VT>
__device__ __forceinline__ int stage_values(const IcholArgs<VT>& a, int j, VT* sval) {
    const int64_t t0 = a.rowptr[j];
    const int np = int(a.rowend[j] - 1 - t0);
    for (int t = threadIdx.x; t < np; t += blockDim.x) sval[t] = a.Lv[t0 + t];
    return np;
}

// factor_entries with match masks: the lane walks row k's values up to its last
// match, and for each set bit of mk takes the next set bit of mj to find L_ji in
// the staged row -- the same updates in the same order as the index merge, from
// one bit per walked entry instead of a 16-bit index gap.  A value piece with
// no set bit is not loaded.  Every loop is bounded by the masks' lengths and
// every read checked against them, so inconsistent masks are counted
// (kMatchErr), never followed outside row j or the mask buffer.
template <int TWONU, bool COUNT, typename VT>
__device__ __forceinline__ void factor_entries_mask(const IcholArgs<VT>& a, int j, int first, int np, int lane,
                                                    const VT* sval) {
    const int64_t* __restrict__ colptr = a.colptr;
    const uint32_t* __restrict__ csc2csr = a.csc2csr;
    VT* __restrict__ Lv = a.Lv;
    const double* __restrict__ xh = a.xh;
    const int d = a.d, policy = a.policy;
    double ell = a.ell;
    unsigned long long* __restrict__ counters = a.counters;

    double dacc = 1.0;  // Theta_jj
    for (int t = 0; t < np; ++t) {
        double v = double(sval[t]);
        dacc = __builtin_fma(-v, v, dacc);
    }

    const int64_t e = colptr[j] + first + lane;
    const bool active = e < colptr[j + 1];
    const int k = active ? a.rowidx[e] : j;
    if (a.ells) ell = a.ells[a.inst[j]];
    int hard = 0;
    VT acc;
    if constexpr (sizeof(VT) == 8)
        acc = kcdev::matern<TWONU>(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d), ell, hard);
    else
        acc = kcdev::matern_f32<TWONU>(float(kcdev::dist(xh + int64_t(k) * d, xh + int64_t(j) * d, d)), float(ell));

    unsigned long long hits = 0;
    bool inconsistent = false;
    if (COUNT && active && k == j) {  // the pivot's own updates A_jj -= L_ji^2, taken from LDS above
        for (int t = 0; t < np; ++t) hits += sval[t] != VT(0);
    }
    if (active && k != j) {
        const int64_t rp = a.rowptr[k];
        const int pos = int(int64_t(csc2csr[e]) - rp);  // row k's entries before (k,j)
        const uint64_t m = a.mmeta[e];
        const uint64_t base = m & kMatchOffMask;
        const int nk = (pos + 63) >> 6, nj = (np + 63) >> 6;
        int wend = int(m >> kMatchOffBits);
        if (base + uint64_t(nk) + uint64_t(nj) > a.mwords_n || wend > pos) {
            inconsistent = true;
            wend = 0;
        }
        const uint64_t* __restrict__ mk = a.mwords + base;
        const uint64_t* __restrict__ mj = mk + nk;
        uint64_t cj = nj > 0 && wend > 0 ? mj[0] : 0, cn = nj > 1 && wend > 0 ? mj[1] : 0;
        int jw = 0;
        constexpr int kPiece = sizeof(VT) == 8 ? 16 : 32;  // values per 128-byte line
        constexpr uint64_t kPieceMask = (uint64_t(1) << kPiece) - 1;
        uint64_t mkn = wend > 0 ? mk[0] : 0;
        for (int w = 0; w * 64 < wend; ++w) {
            const uint64_t mkw = mkn;
            mkn = (w + 1) * 64 < wend ? mk[w + 1] : 0;  // the next window's bits, in flight meanwhile
            const int64_t p = rp + int64_t(w) * 64;
#pragma unroll
            for (int off = 0; off < 64; off += kPiece) {
                const uint64_t bits = (mkw >> off) & kPieceMask;
                if (bits) {
                    VT val[kPiece];
                    load_vals(Lv, p + off, val);
#pragma unroll
                    for (int t = 0; t < kPiece; ++t) {
                        if ((bits >> t) & 1) {
                            while (cj == 0 && jw + 1 < nj) {
                                ++jw;
                                cj = cn;
                                cn = jw + 1 < nj ? mj[jw + 1] : 0;
                            }
                            const int sidx = jw * 64 + (cj ? __builtin_ctzll(cj) : 0);
                            if (cj == 0 || sidx >= np) {
                                inconsistent = true;
                            } else {
                                cj &= cj - 1;
                                const VT lji = sval[sidx];
                                if constexpr (sizeof(VT) == 8) acc = __builtin_fma(-val[t], lji, acc);
                                else acc = __builtin_fmaf(-val[t], lji, acc);
                                if (COUNT && lji != VT(0)) ++hits;
                            }
                        }
                    }
                }
            }
        }
    }

    bool zero = false, shifted = false;
    double piv = dacc;
    if (policy == KC_PIVOT_ZERO) {
        zero = !(piv > 0.0);
    } else {
        const double fl = a.tau * 1.0;
        if (!(piv > fl)) {
            piv = fl;
            shifted = true;
        }
    }
    const double ljj = zero ? 0.0 : __builtin_sqrt(piv);
    bool bad = false;
    if (active) {
        VT out;
        if (zero) out = VT(0);
        else if (k == j) out = VT(ljj);
        else if constexpr (sizeof(VT) == 8) out = acc / ljj;
        else out = float(double(acc) / ljj);
        Lv[csc2csr[e]] = out;
        a.Lcsc[e] = out;
        if constexpr (sizeof(VT) == 4)
            if (k == j) a.diag[j] = ljj;
        bad = !__builtin_isfinite(out);
    }
    const unsigned long long nf = __ballot(bad);
    if (nf && lane == 0) atomicAdd(counters + kNonfinite, (unsigned long long)__popcll(nf));
    const unsigned long long ni = __ballot(inconsistent);
    if (ni && lane == 0) atomicAdd(counters + kMatchErr, (unsigned long long)__popcll(ni));
    if (first == 0 && lane == 0) {
        if (zero) atomicAdd(counters + kNonpos, 1ull);
        if (shifted) atomicAdd(counters + kShifted, 1ull);
    }
    if (COUNT) {
        const unsigned long long tot = wave_sum(hits);
        if (lane == 0 && tot) atomicAdd(counters + kUpdates, tot);
    }
    if (hard && active) atomicAdd(counters + kExpHard, 1ull);
}

// A row j with more parents than a.stage_max (at most a.cap - 2: what the LDS
// holds beside the sentinel) is not staged: its wavefronts read row j's indices
// and values from device memory, where the diagonal entry, index j, ends every
// cursor walk as the sentinel does in LDS -- the same merge, the same updates
// in the same order, so the same L.
template <typename VT>
__device__ __forceinline__ bool row_unstaged(const IcholArgs<VT>& a, int j) {
    return a.rowend[j] - 1 - a.rowptr[j] > a.stage_max;
}

template <int TWONU, bool COUNT, typename VT, bool MASK>
__device__ __forceinline__ void factor_unstaged(const IcholArgs<VT>& a, int j, int first, int lane) {
    const int64_t t0 = a.rowptr[j];
    const int np = int(a.rowend[j] - 1 - t0);
    if (a.colptr[j] + first >= a.colptr[j + 1]) return;
    if constexpr (MASK) factor_entries_mask<TWONU, COUNT, VT>(a, j, first, np, lane, a.Lv + t0);
    else factor_entries<TWONU, COUNT, VT, false>(a, j, first, np, lane, a.Lv + t0, a.colidx + t0, nullptr, 0);
}

// One DAG level per launch.  A workgroup owns a block unit: 64 * WPB consecutive
// entries of one column, 64 per wave, with the column's row staged once in LDS.
// MASK: the factorization with match masks (factor_entries_mask; only the
// values of row j are staged); else the index merge (factor_entries).
template <int TWONU, bool COUNT, typename VT, int WPB, bool MASK>
__global__ __launch_bounds__(WPB * kWave) void ichol_level(IcholArgs<VT> a, const Unit* __restrict__ bunits,
                                                           int64_t ubeg, int64_t uend) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    VT* sval = reinterpret_cast<VT*>(smem);
    int32_t* sidx = reinterpret_cast<int32_t*>(smem + size_t(a.cap) * sizeof(VT));
    uint16_t* sb = reinterpret_cast<uint16_t*>(smem + size_t(a.cap) * (sizeof(VT) + sizeof(int32_t)));
    const int64_t bu = ubeg + int64_t(blockIdx.x);  // longest first (see block_units)
    if (bu >= uend) return;  // the whole workgroup
    const int j = __builtin_amdgcn_readfirstlane(bunits[bu].col);
    const int first = __builtin_amdgcn_readfirstlane(bunits[bu].first) + wave * kWave;
    if (row_unstaged(a, j)) {
        factor_unstaged<TWONU, COUNT, VT, MASK>(a, j, first, lane);
        return;
    }
    if constexpr (MASK) {
        const int np = stage_values(a, j, sval);
        __syncthreads();
        if (a.colptr[j] + first < a.colptr[j + 1]) factor_entries_mask<TWONU, COUNT, VT>(a, j, first, np, lane, sval);
    } else {
        const int np = stage_row(a, j, sval, sidx);
        __syncthreads();
        int shift = 0;
        if (a.nbuck) {
            shift = build_buckets(sidx, np, j, a.nbuck, sb);
            __syncthreads();
        }
        if (a.colptr[j] + first < a.colptr[j + 1]) {
            if (a.nbuck) factor_entries<TWONU, COUNT, VT, true>(a, j, first, np, lane, sval, sidx, sb, shift);
            else factor_entries<TWONU, COUNT, VT, false>(a, j, first, np, lane, sval, sidx, sb, shift);
        }
    }
}

// Levels [l0, l1) in one persistent launch: the workgroups of a grid that is
// resident as a whole (cooperative launch) stride over each level's block units,
// and a grid-wide barrier separates consecutive levels.
template <int TWONU, bool COUNT, typename VT, int WPB, bool MASK>
__global__ __launch_bounds__(WPB * kWave) void ichol_persistent(IcholArgs<VT> a, const Unit* __restrict__ bunits,
                                                                const int64_t* __restrict__ boff, int l0, int l1) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    VT* sval = reinterpret_cast<VT*>(smem);
    int32_t* sidx = reinterpret_cast<int32_t*>(smem + size_t(a.cap) * sizeof(VT));
    uint16_t* sb = reinterpret_cast<uint16_t*>(smem + size_t(a.cap) * (sizeof(VT) + sizeof(int32_t)));
    const int64_t slot = blockIdx.x, stride = gridDim.x;
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    for (int l = l0; l < l1; ++l) {
        const int64_t ub = boff[l], ue = boff[l + 1];
        for (int64_t bu = ub + slot; bu < ue; bu += stride) {  // the same trip count for the whole workgroup
            const int j = __builtin_amdgcn_readfirstlane(bunits[bu].col);
            const int first = __builtin_amdgcn_readfirstlane(bunits[bu].first) + wave * kWave;
            if (row_unstaged(a, j)) {
                factor_unstaged<TWONU, COUNT, VT, MASK>(a, j, first, lane);
                continue;  // no LDS touched: the workgroup needs no barrier before its next unit
            }
            if constexpr (MASK) {
                const int np = stage_values(a, j, sval);
                __syncthreads();
                if (a.colptr[j] + first < a.colptr[j + 1])
                    factor_entries_mask<TWONU, COUNT, VT>(a, j, first, np, lane, sval);
            } else {
                const int np = stage_row(a, j, sval, sidx);
                __syncthreads();
                int shift = 0;
                if (a.nbuck) {
                    shift = build_buckets(sidx, np, j, a.nbuck, sb);
                    __syncthreads();
                }
                if (a.colptr[j] + first < a.colptr[j + 1]) {
                    if (a.nbuck)
                        factor_entries<TWONU, COUNT, VT, true>(a, j, first, np, lane, sval, sidx, sb, shift);
                    else
                        factor_entries<TWONU, COUNT, VT, false>(a, j, first, np, lane, sval, sidx, sb, shift);
                }
            }
            __syncthreads();  // the staged row is free again
        }
        grid.sync();
    }
}

// ---------------------------------------------------------------------------
// Supernodal groups on the matrix cores (mixed precision, supernodal plans).
//
// The block-closed pattern makes every member of a supernode J = [s0, s1) share
// one row structure: row g of a member is P(J) (the parents of s0), then s0..g-1;
// column g is g..s1-1, then the rows O_J of the other supernodes below J.  A
// group G = [g0, g1) of at most 16 consecutive members therefore shares its
// parents P_G = row g0 before its diagonal, and for a row k of column g0 the
// Schur updates of all 16 entries (k, g), g in G, run over the same parents
// i in P_G that row k holds:
//     a_kg = Theta_kg - sum_{i in P_G, i in row k} L_ki L_gi - sum_{g0 <= h < g} L_kh L_gh.
// The first sum, for 64 rows at once, is a dense product (64 x |P_G|) . (|P_G| x 16)
// on v_mfma_f32_16x16x4f32: row k's values are scattered into an LDS tile over
// P_G (row k is walked once for the whole group, instead of once per column as
// in the element-wise kernel) and the group's rows L_{G,P_G} form the other
// operand.  The second sum and the divisions follow in registers, column by
// column: the dense Cholesky of the group's diagonal block with FP64 pivots
// (accumulated as in the element-wise kernel, FP32 x FP32 products exact in
// FP64), then the panel rows.  A unit is one group with its 16 diagonal rows
// (recomputed by every unit of the group, written by the first) and 48 panel
// rows; the units of a level of the group DAG run in one launch.
constexpr int kGroupCols = 16;  // columns of a group: the width of the MFMA tile
constexpr int kGroupRows = 48;  // panel rows of a unit, beside the group's 16 diagonal rows
constexpr int kGroupKC = 64;    // parents per LDS chunk

typedef float mfma_f4 __attribute__((ext_vector_type(4)));

template <int TWONU>
__global__ __launch_bounds__(kWave) void ichol_group(IcholArgs<float> a, const kc::GroupDesc* __restrict__ groups,
                                                     const int2* __restrict__ gunits, int64_t ubeg, int64_t uend) {
    __shared__ float As[kWave][kGroupKC + 1];
    __shared__ float Bs[kGroupCols][kGroupKC + 1];
    __shared__ float Cs[kWave][kGroupCols + 1];
    __shared__ float Ld[kGroupCols][kGroupCols + 1];
    __shared__ double piv[kGroupCols];
    __shared__ int pzero[kGroupCols];
    extern __shared__ __align__(16) unsigned char smem[];
    int32_t* sP = reinterpret_cast<int32_t*>(smem);  // the group's parents, then a sentinel
    const int lane = threadIdx.x;
    const int64_t u = ubeg + int64_t(blockIdx.x);
    if (u >= uend) return;
    const int2 gu = gunits[u];
    const kc::GroupDesc G = groups[gu.x];
    const int tile = gu.y;
    const int g0 = G.g0, m = G.g1 - G.g0;
    const int64_t t0 = a.rowptr[g0];
    const int np = int(a.rowend[g0] - 1 - t0);
    for (int t = lane; t < np; t += kWave) sP[t] = a.colidx[t0 + t];
    if (lane == 0) sP[np] = INT_MAX;
    // this lane's row: lanes 0..15 the group's diagonal rows g0 + lane, lanes 16..63 panel rows
    const int64_t cg0 = a.colptr[g0];
    int k = -1;
    int64_t eoff = -1;  // offset of (k, g0) in column g0
    if (lane < kGroupCols) {
        if (lane < m) {
            k = g0 + lane;
            eoff = lane;
        }
    } else {
        const int64_t pr = int64_t(tile) * kGroupRows + (lane - kGroupCols);
        if (pr < G.nb) {
            eoff = m + pr;
            k = a.rowidx[cg0 + eoff];
        }
    }
    const bool panel = lane >= kGroupCols && k >= 0;
    int64_t p = 0, pend = 0;  // the walk of row k before (k, g0)
    int q = 0;                // cursor over the parents
    if (panel) {
        p = a.rowptr[k];
        pend = a.csc2csr[cg0 + eoff];
    }
    wave_lds_sync();

    mfma_f4 acc[4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) acc[rb] = mfma_f4{0.f, 0.f, 0.f, 0.f};
    double dd = 1.0;  // pivot of diagonal row `lane`: Theta_jj = 1 minus the squares, ascending
    for (int c0 = 0; c0 < np; c0 += kGroupKC) {
        const int cn = np - c0 < kGroupKC ? np - c0 : kGroupKC;
        for (int idx = lane; idx < kGroupCols * kGroupKC; idx += kWave) {
            const int g = idx / kGroupKC, qq = idx % kGroupKC;
            Bs[g][qq] = (g < m && qq < cn) ? a.Lv[a.rowptr[g0 + g] + c0 + qq] : 0.f;
        }
#pragma unroll
        for (int qq = 0; qq < kGroupKC; ++qq) As[lane][qq] = 0.f;
        wave_lds_sync();
        if (lane < m) {  // a diagonal row's prefix is P_G itself
            for (int qq = 0; qq < cn; ++qq) {
                const float v = Bs[lane][qq];
                As[lane][qq] = v;
                dd = __builtin_fma(-double(v), double(v), dd);
            }
        }
        bool more = panel && p < pend;
        while (more) {  // eight entries of row k per load, from an 8-aligned start (rows are 64-aligned)
            const int64_t bp = p & ~int64_t(7);
            const int4 ia = *reinterpret_cast<const int4*>(a.colidx + bp);
            const int4 ib = *reinterpret_cast<const int4*>(a.colidx + bp + 4);
            const float4 va = *reinterpret_cast<const float4*>(a.Lv + bp);
            const float4 vb = *reinterpret_cast<const float4*>(a.Lv + bp + 4);
            const int ii[8] = {ia.x, ia.y, ia.z, ia.w, ib.x, ib.y, ib.z, ib.w};
            const float vv[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};
#pragma unroll
            for (int h = 0; h < 8; ++h) {
                if (more && bp + h >= p) {
                    if (bp + h >= pend) {
                        more = false;
                    } else {
                        const int i = ii[h];
                        while (sP[q] < i) ++q;  // the sentinel stops at np
                        if (q >= c0 + cn) {
                            more = false;  // a later chunk: resume here
                        } else {
                            if (sP[q] == i) As[lane][q - c0] = vv[h];
                            p = bp + h + 1;
                        }
                    }
                }
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int ks = 0; ks < kGroupKC / 4; ++ks) {
            const int kk = ks * 4 + lane / 16, col = lane % 16;
            const float bv = Bs[col][kk];
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
                acc[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(As[rb * 16 + col][kk], bv, acc[rb], 0, 0, 0);
        }
        wave_lds_sync();
    }
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) Cs[rb * 16 + 4 * (lane / 16) + i][lane % 16] = acc[rb][i];
    wave_lds_sync();

    // external part: a_g = Theta_kg - C_kg
    float av[kGroupCols], Lr[kGroupCols];
    double ell = a.ell;
#pragma unroll
    for (int g = 0; g < kGroupCols; ++g) {
        av[g] = 0.f;
        Lr[g] = 0.f;
        if (k >= 0 && g < m && k != g0 + g) {
            const float th = kcdev::matern_f32<TWONU>(
                float(kcdev::dist(a.xh + int64_t(k) * a.d, a.xh + int64_t(g0 + g) * a.d, a.d)), float(ell));
            av[g] = th - Cs[lane][g];
        }
    }
    // the group's columns in order: pivot from diagonal lane g, then the rows below
#pragma unroll
    for (int g = 0; g < kGroupCols; ++g) {
        if (g < m) {
            if (lane == g) {
                double pd = dd;
#pragma unroll
                for (int h = 0; h < g; ++h) pd = __builtin_fma(-double(Lr[h]), double(Lr[h]), pd);
                bool zero = false;
                if (a.policy == KC_PIVOT_ZERO) {
                    zero = !(pd > 0.0);
                } else if (!(pd > a.tau)) {
                    pd = a.tau;
                    if (tile == 0) atomicAdd(a.counters + kShifted, 1ull);
                }
                if (zero && tile == 0) atomicAdd(a.counters + kNonpos, 1ull);
                piv[g] = zero ? 0.0 : __builtin_sqrt(pd);
                pzero[g] = zero;
            }
            wave_lds_sync();
            const double ljj = piv[g];
            const bool zero = pzero[g] != 0;
            if ((lane < m && lane > g) || panel) {
                float x = av[g];
#pragma unroll
                for (int h = 0; h < g; ++h) x = __builtin_fmaf(-Lr[h], Ld[g][h], x);
                Lr[g] = zero ? 0.f : float(double(x) / ljj);
                if (lane < m) Ld[lane][g] = Lr[g];
            }
            wave_lds_sync();
        }
    }
    // write: panel rows by every unit, the diagonal block by the group's first unit
    bool bad = false;
    if (k >= 0 && (panel || tile == 0)) {
#pragma unroll
        for (int g = 0; g < kGroupCols; ++g) {
            if (g < m && (panel || lane >= g)) {
                const int j = g0 + g;
                const int64_t e = k < G.s1 ? a.colptr[j] + (k - j) : a.colptr[j] + (G.s1 - j) + (eoff - (G.s1 - g0));
                const float out = lane == g ? float(piv[g]) : Lr[g];
                a.Lcsc[e] = out;
                a.Lv[a.csc2csr[e]] = out;
                if (lane == g) a.diag[j] = piv[g];
                bad = bad || !__builtin_isfinite(out);
            }
        }
    }
    const unsigned long long nf = __ballot(bad);
    if (nf && lane == 0) atomicAdd(a.counters + kNonfinite, (unsigned long long)__popcll(nf));
}

// ---------------------------------------------------------------------------
// A3: y = L^{-1} P b by rows (forward levels), x = P^T L^{-T} y by columns
// (reverse levels).  A wavefront owns one row (one column): its lanes stage 64
// entries at a time in LDS -- the L values and the gathered right-hand-side
// rows -- and lanes r < NR then apply them to right-hand side r in ascending
// index order, one fma each, exactly the sequential substitution.
//
// Long columns are the coarse ones, and each reverse level near the end holds
// only a few of them: one launch per such level would stream their long row
// lists level after level.  When a column is longer than kLongColumn, the
// columns below T (T = one past the last long column: the top block) are
// instead finished in three stages.  (1) The columns at or above T need only
// rows at or above T, so they are solved first, by reverse level as above.
// (2) All their x are then final, so one launch forms every top column's dot
// product over its rows at or above T, in pieces that each stay inside one band
// of row indices; the pieces go out band after band, so the XCD working on a
// band finds its x rows in its L2.  (3) The top block is solved by its own
// levels: a wavefront per column adds up the column's piece sums and its rows
// below T in a fixed order.  Deterministic, but summed in a different order
// than the sequential substitution.

template <typename VT>
__device__ __forceinline__ double diag_value(const VT* Lv, const double* diag, int64_t pos, int k) {
    if constexpr (sizeof(VT) == 8) return Lv[pos];
    else return diag[k];
}

// Staging of one 64-entry chunk in LDS: sL holds the chunk's L values, sY the
// gathered right-hand-side rows, transposed -- right-hand side r's 64 values
// form one row of kYStride doubles.  Lane e stores entry e of every row (word
// stride 2 between lanes: no bank conflict); lane r < NR later reads its own row
// two entries at a time, and the rows start 4 banks apart, so those 128-bit
// reads do not conflict either.
constexpr int kYStride = kWave + 2;

// acc -= sum_q sL[q] * sY[lane * kYStride + q] for q = 0..m-1 in ascending order
// (the sequential substitution).  LDS reads are issued eight entries at a time,
// as four 128-bit reads of each array, so their latency is paid once per eight
// dependent fmas.
__device__ __forceinline__ double apply_chunk(const double* __restrict__ sL, const double* __restrict__ sY, int m,
                                              int lane, double acc) {
    const double* yr = sY + lane * kYStride;
    int q = 0;
    for (; q + 8 <= m; q += 8) {
        double2 a[4], v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = *reinterpret_cast<const double2*>(sL + q + 2 * u);
            v[u] = *reinterpret_cast<const double2*>(yr + q + 2 * u);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            acc = __builtin_fma(-a[u].x, v[u].x, acc);
            acc = __builtin_fma(-a[u].y, v[u].y, acc);
        }
    }
    for (; q < m; ++q) acc = __builtin_fma(-sL[q], yr[q], acc);
    return acc;
}

// acc - sum over entries p in [b0, b1) of val[p] * src[idx[p]] (one value per
// right-hand side), applied in ascending p by lanes r < NR -- the sequential
// substitution.  The indices and values of kGroup 64-entry chunks are fetched at
// once; then each chunk's gathered right-hand-side rows are requested before the
// previous chunk is applied, so the gathers overlap the dependent fmas.
constexpr int kGroup = 6;  // 384 entries: a whole row of the 2-D benchmark in one fetch

template <int NR>
__device__ __forceinline__ void gather_chunk(const double* __restrict__ src, int ld, int r0, int i, double (&v)[NR]) {
    if (i >= 0) {
        const double* si = src + int64_t(i) * ld + r0;
#pragma unroll
        for (int r = 0; r < NR; ++r) v[r] = si[r];
    }
}

template <typename VT, int NR>
__device__ __forceinline__ double substitute(const int32_t* __restrict__ idx, const VT* __restrict__ val, int64_t b0,
                                             int64_t b1, const double* __restrict__ src, int ld, int r0, int lane,
                                             double* sL, double* sY, double acc) {
    for (int64_t cb = b0; cb < b1; cb += kGroup * kWave) {
        int ci[kGroup];
        double lv[kGroup];
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int64_t p = cb + int64_t(u) * kWave + lane;
            ci[u] = p < b1 ? idx[p] : -1;
            lv[u] = p < b1 ? double(val[p]) : 0.0;
        }
        double yv[2][NR];
        gather_chunk<NR>(src, ld, r0, ci[0], yv[0]);
#pragma unroll
        for (int u = 0; u < kGroup; ++u) {
            const int64_t c = cb + int64_t(u) * kWave;
            if (c >= b1) break;
            if (u + 1 < kGroup) gather_chunk<NR>(src, ld, r0, ci[u + 1 < kGroup ? u + 1 : u], yv[(u + 1) & 1]);
            if (ci[u] >= 0) {
                sL[lane] = lv[u];
#pragma unroll
                for (int r = 0; r < NR; ++r) sY[r * kYStride + lane] = yv[u & 1][r];
            }
            wave_lds_sync();
            if (lane < NR) acc = apply_chunk(sL, sY, int(b1 - c < kWave ? b1 - c : kWave), lane, acc);
            wave_lds_sync();
        }
    }
    return acc;
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void fwd_solve(const int32_t* __restrict__ rows, int64_t beg, int64_t end,
                                                    const int64_t* __restrict__ rowptr,
                                                    const int64_t* __restrict__ rowend,
                                                    const int32_t* __restrict__ colidx, const VT* __restrict__ Lv,
                                                    const double* __restrict__ diag,
                                                    const int32_t* __restrict__ perm, const double* __restrict__ b,
                                                    int ld, int r0, double* __restrict__ y) {
    __shared__ __align__(16) double sL[kWavesPerBlock][kWave];
    __shared__ __align__(16) double sY[kWavesPerBlock][NR * kYStride];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t t = beg + int64_t(xcd_block()) * kWavesPerBlock + wave;
    if (t >= end) return;
    const int k = __builtin_amdgcn_readfirstlane(rows[t]);
    const int64_t p0 = rowptr[k], pd = rowend[k] - 1;  // pd: the diagonal
    double acc = 0.0;
    if (lane < NR) acc = b[int64_t(perm[k]) * ld + r0 + lane];
    // parents' values are final: earlier levels
    acc = substitute<VT, NR>(colidx, Lv, p0, pd, y, ld, r0, lane, sL[wave], sY[wave], acc);
    if (lane < NR) {
        const double lkk = diag_value(Lv, diag, pd, k);
        y[int64_t(k) * ld + r0 + lane] = (lkk == 0.0) ? 0.0 : acc / lkk;
    }
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void bwd_solve(const int32_t* __restrict__ cols, int64_t beg, int64_t end,
                                                    const int64_t* __restrict__ colptr,
                                                    const int32_t* __restrict__ rowidx, const VT* __restrict__ Lcsc,
                                                    const double* __restrict__ diag,
                                                    const int32_t* __restrict__ perm, int ld, int r0,
                                                    double* __restrict__ y, double* __restrict__ x) {
    __shared__ __align__(16) double sL[kWavesPerBlock][kWave];
    __shared__ __align__(16) double sY[kWavesPerBlock][NR * kYStride];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t t = beg + int64_t(xcd_block()) * kWavesPerBlock + wave;
    if (t >= end) return;
    const int j = __builtin_amdgcn_readfirstlane(cols[t]);
    const int64_t c0 = colptr[j], c1 = colptr[j + 1];
    double acc = 0.0;
    if (lane < NR) acc = y[int64_t(j) * ld + r0 + lane];
    // rows below j are final: earlier reverse levels
    acc = substitute<VT, NR>(rowidx, Lcsc, c0 + 1, c1, y, ld, r0, lane, sL[wave], sY[wave], acc);
    if (lane < NR) {
        const double ljj = diag_value(Lcsc, diag, c0, j);
        const double v = (ljj == 0.0) ? 0.0 : acc / ljj;
        y[int64_t(j) * ld + r0 + lane] = v;
        x[int64_t(perm[j]) * ld + r0 + lane] = v;
    }
}

// s[r] += sum of L_e * y[row_e][r] over this lane's entries e = e, e + STRIDE,
// ... below e1, in ascending order: four entries in flight at once, and the row
// indices of the next four requested before this four's values and gathers,
// so each step waits for one round trip instead of two.
template <typename VT, int NR, int STRIDE = kWave>
__device__ __forceinline__ void dot_entries(const int32_t* __restrict__ rowidx, const VT* __restrict__ Lcsc, int64_t e,
                                            int64_t e1, const double* __restrict__ y, int ld, int r0,
                                            double (&s)[NR]) {
    constexpr int kDepth = 4;
    int ci[kDepth];
#pragma unroll
    for (int u = 0; u < kDepth; ++u) {
        const int64_t eu = e + int64_t(u) * STRIDE;
        ci[u] = eu < e1 ? rowidx[eu] : -1;
    }
    for (; e < e1; e += kDepth * STRIDE) {
        int cn[kDepth];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            const int64_t en = e + int64_t(kDepth + u) * STRIDE;
            cn[u] = en < e1 ? rowidx[en] : -1;
        }
        double l[kDepth], v[kDepth][NR];
#pragma unroll
        for (int u = 0; u < kDepth; ++u) {
            l[u] = 0.0;
            if (ci[u] >= 0) {
                l[u] = double(Lcsc[e + int64_t(u) * STRIDE]);
                const double* xk = y + int64_t(ci[u]) * ld + r0;
#pragma unroll
                for (int r = 0; r < NR; ++r) v[u][r] = xk[r];
            }
        }
#pragma unroll
        for (int u = 0; u < kDepth; ++u)
            if (ci[u] >= 0) {
#pragma unroll
                for (int r = 0; r < NR; ++r) s[r] = __builtin_fma(l[u], v[u][r], s[r]);
            }
#pragma unroll
        for (int u = 0; u < kDepth; ++u) ci[u] = cn[u];
    }
}

// Partial dot products of column pieces: one wavefront per piece.
template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void bwd_partial(const kc::BwdChunk* __restrict__ chunks, int64_t beg,
                                                      int64_t end, const int64_t* __restrict__ colptr,
                                                      const int32_t* __restrict__ rowidx,
                                                      const VT* __restrict__ Lcsc, int ld, int r0,
                                                      const double* __restrict__ y, double* __restrict__ partial) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t t = beg + int64_t(xcd_block()) * kWavesPerBlock + wave;
    if (t >= end) return;
    const kc::BwdChunk ch = chunks[t];
    const int64_t e0 = colptr[ch.col] + 1 + ch.start;
    const int64_t e1 = e0 + ch.len;
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    dot_entries<VT, NR>(rowidx, Lcsc, e0 + lane, e1, y, ld, r0, s);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s[r] += __shfl_xor(s[r], off, kWave);
    if (lane < NR) {
        double v = s[0];
#pragma unroll
        for (int r = 1; r < NR; ++r)
            if (lane == r) v = s[r];
        partial[int64_t(ch.slot) * NR + lane] = v;
    }
}

// Forward levels of at least kWideRows rows: there a wavefront's 64 lanes share
// a row's dot product (every 64th entry, four in flight) and a fixed butterfly
// adds them, instead of 8 lanes applying staged chunks in the sequential
// order -- more throughput on large levels and a shorter chain per row on
// medium ones.  Deterministic, but not the sequential substitution's
// summation order; smaller levels keep that order.
constexpr int64_t kWideRows = 1024;

template <typename VT, int NR>
__device__ __forceinline__ double wave_dot(const int32_t* __restrict__ idx, const VT* __restrict__ val, int64_t b0,
                                           int64_t b1, const double* __restrict__ src, int ld, int r0, int lane) {
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    dot_entries<VT, NR>(idx, val, b0 + lane, b1, src, ld, r0, s);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s[r] += __shfl_xor(s[r], off, kWave);
    double v = s[0];
#pragma unroll
    for (int r = 1; r < NR; ++r)
        if (lane == r) v = s[r];
    return v;  // lane r < NR holds right-hand side r's sum
}

template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void fwd_wide(const int32_t* __restrict__ rows, int64_t beg, int64_t end,
                                                   const int64_t* __restrict__ rowptr,
                                                   const int64_t* __restrict__ rowend,
                                                   const int32_t* __restrict__ colidx, const VT* __restrict__ Lv,
                                                   const double* __restrict__ diag, const int32_t* __restrict__ perm,
                                                   const double* __restrict__ b, int ld, int r0,
                                                   double* __restrict__ y) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t t = beg + int64_t(xcd_block()) * kWavesPerBlock + wave;
    if (t >= end) return;
    const int k = __builtin_amdgcn_readfirstlane(rows[t]);
    const int64_t p0 = rowptr[k], pd = rowend[k] - 1;  // pd: the diagonal
    const double v = wave_dot<VT, NR>(colidx, Lv, p0, pd, y, ld, r0, lane);
    if (lane < NR) {
        const double lkk = diag_value(Lv, diag, pd, k);
        const double acc = b[int64_t(perm[k]) * ld + r0 + lane] - v;
        y[int64_t(k) * ld + r0 + lane] = (lkk == 0.0) ? 0.0 : acc / lkk;
    }
}

// Completes the top columns of one top level: a workgroup per column.  Its
// threads add the column's piece sums (thread t takes every kBlock-th slot)
// and, for a short top part, its entries (every kBlock-th, four in flight);
// each wavefront reduces by a fixed butterfly, and the four wavefront sums are
// added in wavefront order; x_j = (y_j - sum) / L_jj.
template <typename VT, int NR>
__global__ __launch_bounds__(kBlock) void bwd_finish(const kc::TopCol* __restrict__ tcols, int64_t beg, int64_t end,
                                                     const int64_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ rowidx,
                                                     const VT* __restrict__ Lcsc, const double* __restrict__ diag,
                                                     const int32_t* __restrict__ perm, int ld, int r0,
                                                     const double* __restrict__ partial, double* __restrict__ y,
                                                     double* __restrict__ x) {
    __shared__ double wsum[kWavesPerBlock][NR];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = threadIdx.x % kWave;
    const int64_t t = beg + int64_t(xcd_block());
    if (t >= end) return;  // the whole workgroup
    const kc::TopCol tc = tcols[t];
    const int tid = int(threadIdx.x);
    double s[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) s[r] = 0.0;
    for (int q = tid; q < tc.n1; q += kBlock) {
        const double* pq = partial + int64_t(tc.s1 + q) * NR;
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += pq[r];
    }
    for (int q = tid; q < tc.n2; q += kBlock) {
        const double* pq = partial + int64_t(tc.s2 + q) * NR;
#pragma unroll
        for (int r = 0; r < NR; ++r) s[r] += pq[r];
    }
    const int64_t c0 = colptr[tc.col];
    if (tc.n2 == 0)  // rows of the top part: their columns lie in earlier top levels
        dot_entries<VT, NR, kBlock>(rowidx, Lcsc, c0 + 1 + tid, c0 + 1 + tc.ntop, y, ld, r0, s);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) s[r] += __shfl_xor(s[r], off, kWave);
    if (lane < NR) {
        double v = s[0];
#pragma unroll
        for (int r = 1; r < NR; ++r)
            if (lane == r) v = s[r];
        wsum[wave][lane] = v;
    }
    __syncthreads();
    if (wave == 0 && lane < NR) {
        double v = wsum[0][lane];
#pragma unroll
        for (int w = 1; w < kWavesPerBlock; ++w) v += wsum[w][lane];
        const double ljj = diag_value(Lcsc, diag, c0, tc.col);
        double* yj = y + int64_t(tc.col) * ld + r0 + lane;
        const double xv = (ljj == 0.0) ? 0.0 : (*yj - v) / ljj;
        *yj = xv;
        x[int64_t(perm[tc.col]) * ld + r0 + lane] = xv;
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


namespace {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

struct BwdSchedule {
    int32_t top = 0;                      // the largest T (0: no long column in any instance)
    std::vector<int32_t> shortc;          // columns >= T by reverse level
    std::vector<int64_t> short_off;
    std::vector<kc::BwdChunk> chunks;     // the nfine band-major pieces, then the long top parts' pieces
    int64_t nfine = 0;
    std::vector<kc::TopCol> topc;         // columns < T by top level
    std::vector<int64_t> top_off, tchunk_off;
    int64_t max_slots = 0;
};

// The backward sweep's schedule (see the A3 kernels), per instance of a batch
// plan (a single problem is one instance) and merged across instances by level:
// the columns at or above the instance's T by reverse level; the pieces of its
// top columns' rows at or above T, each within one band of row indices (bands
// of at most kBandRows over [T, end of the instance)), band after band; the
// top block by its own levels (a column's level is one more than the highest
// level among the rows of its top part).
BwdSchedule backward_schedule(const kc::Plan& p) {
    BwdSchedule b;
    const int32_t n = p.n;
    const int32_t ni = std::max<int32_t>(1, p.ninst);
    auto inst_begin = [&](int32_t i) -> int32_t { return ni == 1 ? 0 : int32_t(p.inst_off[size_t(i)]); };
    auto inst_end = [&](int32_t i) -> int32_t { return ni == 1 ? n : int32_t(p.inst_off[size_t(i) + 1]); };
    // T of each instance: one past its last long column (its first position: no top block)
    std::vector<int32_t> tops(static_cast<size_t>(ni));
    for (int32_t i = 0; i < ni; ++i) {
        int32_t t = inst_begin(i);
        for (int32_t j = inst_begin(i); j < inst_end(i); ++j)
            if (p.colptr[j + 1] - p.colptr[j] - 1 > kLongColumn) t = j + 1;
        tops[size_t(i)] = t;
        if (t > inst_begin(i)) b.top = std::max(b.top, t);
    }
    auto top_of = [&](int32_t j) { return tops[size_t(ni == 1 ? 0 : p.inst[size_t(j)])]; };
    const int32_t nl = p.nrlevels;
    b.short_off.assign(size_t(nl + 1), 0);
    for (int32_t v = 0; v < nl; ++v) {
        for (int64_t q = p.bwd_off[v]; q < p.bwd_off[v + 1]; ++q) {
            const int32_t j = p.bwd_cols[size_t(q)];
            if (j >= top_of(j)) b.shortc.push_back(j);
        }
        b.short_off[v + 1] = int64_t(b.shortc.size());
    }
    if (b.top == 0) return b;
    // top columns: entries [c0 + 1, fb) have rows < T of the instance, [fb, c1) rows >= T
    std::vector<int64_t> fb(static_cast<size_t>(n), 0);
    std::vector<int32_t> s1(static_cast<size_t>(n), 0), n1(static_cast<size_t>(n), 0);
    int64_t slot = 0;
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t i0 = inst_begin(i), T = tops[size_t(i)], iend = inst_end(i);
        if (T == i0) continue;
        for (int32_t j = i0; j < T; ++j)
            fb[size_t(j)] = std::lower_bound(p.rowidx.begin() + p.colptr[j] + 1, p.rowidx.begin() + p.colptr[j + 1], T) -
                            p.rowidx.begin();
        // pieces of the rows >= T: slots column by column, pieces band after band
        const int64_t nfine_rows = int64_t(iend) - T;
        const int64_t nb = std::min<int64_t>(64, std::max<int64_t>(1, (nfine_rows + kBandRows - 1) / kBandRows));
        const int64_t width = std::max<int64_t>(1, (nfine_rows + nb - 1) / nb);
        std::vector<std::vector<kc::BwdChunk>> band(static_cast<size_t>(nb));
        for (int32_t j = i0; j < T; ++j) {
            const int64_t c0 = p.colptr[j], c1 = p.colptr[j + 1];
            s1[size_t(j)] = int32_t(slot);
            int64_t pos = fb[size_t(j)];
            for (int64_t q = 0; q < nb && pos < c1; ++q) {
                const int64_t bound = std::min<int64_t>(int64_t(iend), T + (q + 1) * width);
                const int64_t hi = std::lower_bound(p.rowidx.begin() + pos, p.rowidx.begin() + c1, int32_t(bound)) -
                                   p.rowidx.begin();
                for (int64_t e = pos; e < hi; e += kFinePiece) {
                    const int64_t len = std::min<int64_t>(kFinePiece, hi - e);
                    band[size_t(q)].push_back(kc::BwdChunk{j, int32_t(e - c0 - 1), int32_t(slot++), int32_t(len)});
                }
                pos = hi;
            }
            n1[size_t(j)] = int32_t(slot - s1[size_t(j)]);
        }
        for (auto& bq : band) b.chunks.insert(b.chunks.end(), bq.begin(), bq.end());
    }
    b.nfine = int64_t(b.chunks.size());
    const int64_t fine_slots = slot;
    b.max_slots = fine_slots;
    // levels of the top blocks, merged across instances
    std::vector<int32_t> rt(static_cast<size_t>(n), -1);
    int32_t ntl = 0;
    for (int32_t i = 0; i < ni; ++i) {
        const int32_t i0 = inst_begin(i), T = tops[size_t(i)];
        for (int32_t j = T - 1; j >= i0; --j) {
            int32_t m = -1;
            for (int64_t e = p.colptr[j] + 1; e < fb[size_t(j)]; ++e) m = std::max(m, rt[size_t(p.rowidx[e])]);
            rt[size_t(j)] = m + 1;
            ntl = std::max(ntl, m + 2);
        }
    }
    std::vector<int64_t> cnt(size_t(ntl) + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        if (rt[size_t(j)] >= 0) ++cnt[size_t(rt[size_t(j)]) + 1];
    for (int32_t v = 0; v < ntl; ++v) cnt[size_t(v) + 1] += cnt[size_t(v)];
    std::vector<int32_t> bylevel(static_cast<size_t>(cnt[size_t(ntl)]));
    {
        std::vector<int64_t> at(cnt.begin(), cnt.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            if (rt[size_t(j)] >= 0) bylevel[size_t(at[size_t(rt[size_t(j)])]++)] = j;
    }
    b.top_off.assign(size_t(ntl) + 1, 0);
    b.tchunk_off.assign(size_t(ntl) + 1, 0);
    for (int32_t v = 0; v < ntl; ++v) {
        int64_t lslot = fine_slots;
        for (int64_t q = cnt[size_t(v)]; q < cnt[size_t(v) + 1]; ++q) {
            const int32_t j = bylevel[size_t(q)];
            const int64_t ntop = fb[size_t(j)] - p.colptr[j] - 1;
            kc::TopCol tc{j, s1[size_t(j)], n1[size_t(j)], 0, 0, int32_t(ntop), 0, 0};
            if (ntop > kLongColumn) {
                tc.s2 = int32_t(lslot);
                for (int64_t e = 0; e < ntop; e += kChunk)
                    b.chunks.push_back(
                        kc::BwdChunk{j, int32_t(e), int32_t(lslot++), int32_t(std::min<int64_t>(kChunk, ntop - e))});
                tc.n2 = int32_t(lslot - tc.s2);
            }
            b.topc.push_back(tc);
        }
        b.max_slots = std::max(b.max_slots, lslot);
        b.top_off[size_t(v) + 1] = int64_t(b.topc.size());
        b.tchunk_off[size_t(v) + 1] = int64_t(b.chunks.size()) - b.nfine;
    }
    return b;
}

// Groups of a supernodal plan (see ichol_group) and their units, grouped by the
// level of the group DAG: a group waits for the groups holding its parents.
struct GroupSchedule {
    std::vector<kc::GroupDesc> groups;
    std::vector<int2> units;     // (group, tile of kGroupRows panel rows)
    std::vector<int64_t> off;    // units of each level
};

GroupSchedule group_schedule(const kc::Plan& p) {
    GroupSchedule gs;
    if (p.snode_ptr.empty()) return gs;
    const int64_t n = p.n;
    std::vector<int32_t> gid(static_cast<size_t>(n));
    for (size_t s = 0; s + 1 < p.snode_ptr.size(); ++s) {
        const int32_t s0 = int32_t(p.snode_ptr[s]), s1 = int32_t(p.snode_ptr[s + 1]);
        for (int32_t g0 = s0; g0 < s1; g0 += kGroupCols) {
            const int32_t g1 = std::min(g0 + kGroupCols, s1);
            const int32_t nb = int32_t(p.colptr[size_t(g0) + 1] - p.colptr[size_t(g0)]) - (g1 - g0);
            for (int32_t c = g0; c < g1; ++c) gid[size_t(c)] = int32_t(gs.groups.size());
            gs.groups.push_back(kc::GroupDesc{g0, g1, s1, nb});
        }
    }
    const size_t ng = gs.groups.size();
    std::vector<int32_t> level(ng, 0);
    int32_t nl = 0;
    for (size_t g = 0; g < ng; ++g) {
        const int32_t g0 = gs.groups[g].g0;
        int32_t lv = 0;
        for (int64_t t = p.rowptr[size_t(g0)]; t < p.rowend[size_t(g0)] - 1; ++t)
            lv = std::max(lv, level[size_t(gid[size_t(p.colidx[size_t(t)])])] + 1);
        level[g] = lv;
        nl = std::max(nl, lv + 1);
    }
    gs.off.assign(size_t(nl) + 1, 0);
    for (size_t g = 0; g < ng; ++g) {
        const int32_t nt = std::max(1, (gs.groups[g].nb + kGroupRows - 1) / kGroupRows);
        gs.off[size_t(level[g]) + 1] += nt;
    }
    for (int32_t v = 0; v < nl; ++v) gs.off[size_t(v) + 1] += gs.off[size_t(v)];
    gs.units.resize(size_t(gs.off[size_t(nl)]));
    std::vector<int64_t> fill(gs.off.begin(), gs.off.end() - 1);
    for (size_t g = 0; g < ng; ++g) {
        const int32_t nt = std::max(1, (gs.groups[g].nb + kGroupRows - 1) / kGroupRows);
        for (int32_t t = 0; t < nt; ++t) gs.units[size_t(fill[size_t(level[g])]++)] = int2{int32_t(g), t};
    }
    return gs;
}

struct Layout {
    size_t counters, xh, perm, colptr, rowidx, csc2csr, rowptr, rowend, colidx, cdelta, escptr, esc, L, Lcsc, diag,
        units, unit_off, bunits[2][3], boff[3], fwd, bshort,
        blong, bchunks, inst, groups, gunits, total;
};

Layout layout_of(const kc::Plan& p, const BwdSchedule& b, kc_prec prec, const GroupSchedule& gs = GroupSchedule()) {
    Layout o{};
    size_t at = 0;
    auto take = [&](size_t bytes) {
        size_t r = at;
        at = align256(at + bytes);
        return r;
    };
    const size_t n = size_t(p.n), nnz = size_t(p.nnz()), nnzr = size_t(p.nnz_rows());
    const size_t vt = prec == KC_FP64 ? sizeof(double) : sizeof(float);
    o.counters = take(kNumCounters * sizeof(unsigned long long));
    o.xh = take(n * p.d * sizeof(double));
    o.perm = take(n * sizeof(int32_t));
    o.colptr = take((n + 1) * sizeof(int64_t));
    o.rowidx = take(nnz * sizeof(int32_t));
    o.csc2csr = take(nnz * sizeof(uint32_t));
    o.rowptr = take((n + 1) * sizeof(int64_t));
    o.rowend = take(n * sizeof(int64_t));
    o.colidx = take(nnzr * sizeof(int32_t));
    o.cdelta = take(nnzr * sizeof(uint16_t));
    o.escptr = take((n + 1) * sizeof(uint32_t));
    o.esc = take(std::max<size_t>(p.esc.size(), 1) * sizeof(int32_t));
    o.L = take(nnzr * vt);
    o.Lcsc = take(nnz * vt);
    o.diag = take(prec == KC_FP64 ? 0 : n * sizeof(double));
    o.units = take(p.units.size() * sizeof(Unit));
    o.unit_off = take((size_t(p.nlevels) + 1) * sizeof(int64_t));
    for (int w = 0; w < 3; ++w) {
        const int per = kWave << w;
        size_t nb = 0;
        for (const Unit& u : p.units) nb += (u.first % per == 0);
        for (int r = 0; r < 2; ++r) o.bunits[r][w] = take(nb * sizeof(Unit));
        o.boff[w] = take((size_t(p.nlevels) + 1) * sizeof(int64_t));
    }
    o.fwd = take(n * sizeof(int32_t));
    o.bshort = take(b.shortc.size() * sizeof(int32_t));
    o.blong = take(b.topc.size() * sizeof(kc::TopCol));
    o.bchunks = take(b.chunks.size() * sizeof(kc::BwdChunk));
    o.inst = take(p.ninst > 1 ? n * sizeof(int32_t) : 0);
    o.groups = take(prec == KC_MIXED ? gs.groups.size() * sizeof(kc::GroupDesc) : 0);
    o.gunits = take(prec == KC_MIXED ? gs.units.size() * sizeof(int2) : 0);
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

// LDS entries per wavefront for staging row j (its parents plus a sentinel).
int wpb_slot(int wpb) { return wpb == 4 ? 2 : wpb == 2 ? 1 : 0; }

// Block units for `wpb` wavefronts per workgroup from the plan's 64-entry units
// (each column's units are consecutive and start at entry 0).
// 8 wavefronts per SIMD of the device: the unit of level size in the choices
// below (the factorization kernel itself holds fewer, 5 per SIMD in FP64).
int64_t waves_at_8_per_simd(int num_cu) { return int64_t(std::max(1, num_cu)) * 4 * 8; }

// Runs fn(v) for every level v, the levels handed out one at a time to up to 16
// threads (one thread for small plans).  fn may throw std::bad_alloc, which is
// rethrown here.
template <typename Fn>
void for_levels(int32_t nlevels, bool parallel, Fn fn) {
    const int nt = parallel ? int(std::min(16u, std::max(1u, std::thread::hardware_concurrency()))) : 1;
    std::atomic<int32_t> next{0};
    std::atomic<bool> failed{false};
    auto work = [&]() {
        try {
            for (int32_t v; !failed.load() && (v = next.fetch_add(1)) < nlevels;) fn(v);
        } catch (const std::bad_alloc&) {
            failed = true;
        }
    };
    std::vector<std::thread> pool;
    try {
        for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    } catch (const std::system_error&) {
        // fewer helpers: the calling thread takes whatever levels are left
    }
    work();
    for (auto& th : pool) th.join();
    if (failed) throw std::bad_alloc();
}

// The longest walk of each work unit (64 entries of a column): the longest
// prefix of row k before (k,j) over its entries.  A wavefront lasts about as
// long as its longest lane.  Throws std::bad_alloc.
bool big_plan(const kc::Plan& p) { return p.nnz() >= (int64_t(1) << 22); }

std::vector<int32_t> unit_walks(const kc::Plan& p) {
    std::vector<int32_t> walk(p.units.size());
    for_levels(p.nlevels, big_plan(p), [&](int32_t v) {
        for (int64_t u = p.unit_off[size_t(v)]; u < p.unit_off[size_t(v) + 1]; ++u) {
            const Unit un = p.units[size_t(u)];
            const int64_t e0 = p.colptr[size_t(un.col)] + un.first;
            const int64_t e1 = std::min<int64_t>(e0 + kWave, p.colptr[size_t(un.col) + 1]);
            int64_t w = 0;
            for (int64_t e = e0; e < e1; ++e)
                w = std::max<int64_t>(w, int64_t(p.csc2csr[size_t(e)]) - p.rowptr[size_t(p.rowidx[size_t(e)])]);
            walk[size_t(u)] = int32_t(std::min<int64_t>(w, INT32_MAX));
        }
    });
    return walk;
}

// Block units of each level in one of two orders (results are the same in both;
// only the time differs).  Launches take them in plain block order.
//  - KC_ORDER_SPATIAL: the plan's spatial (k-d tree) order, permuted so that the
//    round-robin dealing of blocks gives each XCD one contiguous slice of the
//    level (the map of xcd_block), whose L2 then serves one region of the points.
//  - KC_ORDER_LONGEST: longest walk first (`walk` from unit_walks; a block unit
//    takes the longest of its wavefronts).  A workgroup lasts as long as its
//    longest lane and workgroups start in index order, so the last, partly
//    filled round of a level then holds the short units.  This pays for a single
//    large problem (10^6-point grid: 146.9 -> 138.7 ms in FP64); a batch of small
//    problems loses more L2 reuse than it gains.
// Throws std::bad_alloc.
void block_units(const std::vector<Unit>& units, const std::vector<int64_t>& unit_off, bool parallel, int wpb,
                 int order, const std::vector<int32_t>& walk, std::vector<Unit>& bu, std::vector<int64_t>& off) {
    const int per = kWave * wpb;
    const int32_t nlevels = int32_t(unit_off.size()) - 1;
    std::vector<int32_t> key;
    bu.clear();
    off.assign(size_t(nlevels) + 1, 0);
    for (int32_t v = 0; v < nlevels; ++v) {
        for (int64_t u = unit_off[size_t(v)]; u < unit_off[size_t(v) + 1]; ++u) {
            const Unit un = units[size_t(u)];
            const int32_t w = order == KC_ORDER_LONGEST ? walk[size_t(u)] : 0;
            if (un.first % per == 0) {
                bu.push_back(un);
                key.push_back(w);
            } else if (!bu.empty() && bu.back().col == un.col) {
                key.back() = std::max(key.back(), w);  // a later wavefront of the same block unit
            }
        }
        off[size_t(v) + 1] = int64_t(bu.size());
    }
    for_levels(nlevels, parallel, [&](int32_t v) {
        const int64_t b0 = off[size_t(v)], b1 = off[size_t(v) + 1], nb = b1 - b0;
        std::vector<std::pair<int32_t, Unit>> lvl;
        lvl.reserve(size_t(nb));
        for (int64_t t = b0; t < b1; ++t) lvl.push_back({key[size_t(t)], bu[size_t(t)]});
        if (order == KC_ORDER_LONGEST) {
            std::stable_sort(lvl.begin(), lvl.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
            for (int64_t t = 0; t < nb; ++t) bu[size_t(b0 + t)] = lvl[size_t(t)].second;
        } else {
            const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
            for (int64_t b = 0; b < nb; ++b) {
                const int64_t x = b % kNumXcd, i = b / kNumXcd;
                bu[size_t(b0 + b)] = lvl[size_t(x * q + std::min<int64_t>(x, r) + i)].second;
            }
        }
    });
}

// Whether the unit order can matter at all: only a level with more units than
// the device holds at once has a last, partly filled round (8 per SIMD bounds
// what it holds).
bool order_matters(const kc::Plan& p, int num_cu) {
    for (int32_t v = 0; v < p.nlevels; ++v)
        if (p.unit_off[size_t(v) + 1] - p.unit_off[size_t(v)] > waves_at_8_per_simd(num_cu)) return true;
    return false;
}

// The default unit order.  SPATIAL when no level exceeds what the device holds
// at once (order cannot matter) and for batches: the units of one small problem
// then stay together, and its rows are reused from L2 (the 512-problem batch:
// 112.5 ms spatial, 121.0 ms longest first).  LONGEST for a single problem,
// whose units of one level lie far apart by construction, so balance wins (the
// jittered grid: 146.9 -> 138.7 ms at 10^6 points, 1020.8 -> 968.6 ms at 4e6).
int32_t default_order(const kc::Plan& p, int num_cu) {
    if (!order_matters(p, num_cu) || p.ninst > 1) return KC_ORDER_SPATIAL;
    return KC_ORDER_LONGEST;
}

// The LONGEST unit order of a factor created with both orders sharing SPATIAL's
// arrays (no level exceeds what the device holds at once, so the order cannot
// change the speed): the unit walks from a device pass over the pattern, sorted
// on the host as block_units does, into the LONGEST region of the workspace.
// Synchronous on s.
kc_status build_longest(kc_factor* f, hipStream_t s) {
    if (f->bunits[KC_ORDER_LONGEST][0] != f->bunits[KC_ORDER_SPATIAL][0]) return KC_OK;  // already built
    const int64_t nu = f->nunits;
    std::vector<Unit> units;
    std::vector<int32_t> walk;
    try {
        units.resize(size_t(nu));
        walk.resize(size_t(nu));
    } catch (const std::bad_alloc&) {
        return KC_ENOMEM;
    }
    if (nu > 0) {
        // the LONGEST region for one wavefront per block holds nunits units: room for the walks
        int32_t* wdev = reinterpret_cast<int32_t*>(f->bunits_alt[0]);
        unit_walk_kernel<<<grid_for(nu, kWavesPerBlock), kBlock, 0, s>>>(f->units, nu, f->colptr, f->rowidx,
                                                                         f->csc2csr, f->rowptr, wdev);
        KC_LAUNCH_CHECK();
        KC_HIP(hipMemcpyAsync(walk.data(), wdev, size_t(nu) * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        KC_HIP(hipMemcpyAsync(units.data(), f->units, size_t(nu) * sizeof(Unit), hipMemcpyDeviceToHost, s));
        KC_HIP(hipStreamSynchronize(s));
    }
    for (int w = 0; w < 3; ++w) {
        std::vector<Unit> bu;
        std::vector<int64_t> off;
        try {
            block_units(units, f->unit_off, nu >= (int64_t(1) << 16), 1 << w, KC_ORDER_LONGEST, walk, bu, off);
        } catch (const std::bad_alloc&) {
            return KC_ENOMEM;
        }
        if (off != f->boff[w]) {
            kc::set_error("build_longest: block units differ from the factor's level offsets");
            return KC_ESTATE;
        }
        if (!bu.empty())
            KC_HIP(hipMemcpyAsync(f->bunits_alt[w], bu.data(), bu.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
        KC_HIP(hipStreamSynchronize(s));  // bu is a local buffer
    }
    for (int w = 0; w < 3; ++w) f->bunits[KC_ORDER_LONGEST][w] = f->bunits_alt[w];
    return KC_OK;
}

int32_t lds_cap(const kc::Plan& p) { return int32_t((p.max_row + 2 + 15) / 16 * 16); }

// Rows longer than this get a bucket directory (the cursor merge costs one
// dependent LDS read per step; fine for short rows, slow for long ones).
constexpr int64_t kBucketRows = 512;
int32_t bucket_count(const kc::Plan& p) {
    if (p.max_row <= kBucketRows) return 0;
    int32_t nb = 1;
    while (nb < 2 * p.max_row && nb < 8192) nb <<= 1;
    return nb;
}

// LDS of a factorization workgroup: the staged row's values, plus its indices and
// bucket directory for the index merge (none with match masks).
size_t factor_lds(const kc_factor* f, size_t vt, bool mask) {
    if (mask) return (size_t(f->cap) * vt + 15) / 16 * 16;
    return (size_t(f->cap) * (vt + sizeof(int32_t)) + (f->nbuck ? size_t(f->nbuck + 1) * sizeof(uint16_t) : 0) + 15) /
           16 * 16;
}
size_t factor_lds(const kc_factor* f, size_t vt) { return factor_lds(f, vt, f->mmeta != nullptr); }

constexpr size_t kMaxLdsBytes = 160 * 1024;

template <typename VT>
IcholArgs<VT> ichol_args(const kc_factor* f, double ell, const double* ells, int pol, double tau) {
    IcholArgs<VT> a;
    a.colptr = f->colptr;
    a.rowidx = f->rowidx;
    a.csc2csr = f->csc2csr;
    a.rowptr = f->rowptr;
    a.rowend = f->rowend;
    a.colidx = f->colidx;
    a.cdelta = f->cdelta;
    a.escptr = f->escptr;
    a.esc = f->esc;
    a.Lv = static_cast<VT*>(f->L);
    a.Lcsc = static_cast<VT*>(f->Lcsc);
    a.diag = f->diag;
    a.xh = f->xh;
    a.d = f->d;
    a.ell = ell;
    a.inst = f->inst;
    a.ells = ells;
    a.policy = pol;
    a.tau = tau;
    a.cap = f->cap;
    a.stage_max = f->stage_max;
    a.nbuck = f->nbuck;
    a.counters = f->counters;
    a.mmeta = f->mmeta;
    a.mwords = f->mwords;
    a.mwords_n = f->mwords_n;
    return a;
}

// One level (block units [ub, ue)) as its own launch, or levels [l0, l1) (at
// most maxb block units each) as one cooperative persistent launch.
template <int TN, bool C, typename VT, int WPB, bool MASK>
kc_status launch_one(const kc_factor* f, const IcholArgs<VT>& a, int64_t ub, int64_t ue, int l0, int l1,
                     int64_t maxb, bool persistent, hipStream_t s) {
    const size_t lds = factor_lds(f, sizeof(VT), MASK);
    const int w = wpb_slot(WPB);
    if (!persistent) {
        if (ue <= ub) return KC_OK;
        ichol_level<TN, C, VT, WPB, MASK><<<unsigned(ue - ub), WPB * kWave, lds, s>>>(a, f->bunits[f->order][w], ub, ue);
        KC_LAUNCH_CHECK();
        return KC_OK;
    }
    const void* fn = reinterpret_cast<const void*>(&ichol_persistent<TN, C, VT, WPB, MASK>);
    int per_cu = 0;
    KC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, WPB * kWave, lds));
    if (per_cu < 1) {
        kc::set_error("kc_factorize: the persistent kernel does not fit on a compute unit");
        return KC_EHIP;
    }
    // every workgroup resident at once (the cooperative launch refuses anything larger)
    const unsigned blocks = unsigned(std::min<int64_t>(int64_t(per_cu) * f->num_cu, std::max<int64_t>(1, maxb)));
    IcholArgs<VT> av = a;
    const Unit* bu = f->bunits[f->order][w];
    const int64_t* bo = f->boff_dev[w];
    int l0v = l0, l1v = l1;
    void* args[] = {&av, &bu, &bo, &l0v, &l1v};
    KC_HIP(hipLaunchCooperativeKernel(fn, dim3(blocks), dim3(WPB * kWave), args, unsigned(lds), s));
    return KC_OK;
}

template <int TN, bool C, typename VT, bool MASK>
kc_status launch_wpb(const kc_factor* f, const IcholArgs<VT>& a, int64_t ub, int64_t ue, int l0, int l1, int64_t maxu,
                     bool persistent, hipStream_t s) {
    if (f->wpb == 4) return launch_one<TN, C, VT, 4, MASK>(f, a, ub, ue, l0, l1, maxu, persistent, s);
    if (f->wpb == 2) return launch_one<TN, C, VT, 2, MASK>(f, a, ub, ue, l0, l1, maxu, persistent, s);
    return launch_one<TN, C, VT, 1, MASK>(f, a, ub, ue, l0, l1, maxu, persistent, s);
}

template <int TN, bool C, typename VT>
kc_status launch_mask(const kc_factor* f, const IcholArgs<VT>& a, int64_t ub, int64_t ue, int l0, int l1,
                      int64_t maxu, bool persistent, hipStream_t s) {
    if (a.mmeta) return launch_wpb<TN, C, VT, true>(f, a, ub, ue, l0, l1, maxu, persistent, s);
    return launch_wpb<TN, C, VT, false>(f, a, ub, ue, l0, l1, maxu, persistent, s);
}

struct NoAfter {
    kc_status operator()(int, int) const { return KC_OK; }
};

// The levels of the factorization: a level with more than f->persist_max units is
// its own launch; each run of consecutive smaller levels is one persistent launch.
// after(l0, l1) is called once the launch covering levels [l0, l1) is enqueued.
template <typename VT, typename After = NoAfter>
kc_status launch_levels(const kc_factor* f, int tn, bool cnt, double ell, const double* ells, int pol, double tau,
                        hipStream_t s, After after = After()) {
    const IcholArgs<VT> a = ichol_args<VT>(f, ell, ells, pol, tau);
    auto go = [&](int64_t ub, int64_t ue, int l0, int l1, int64_t maxu, bool persistent) {
        if (cnt) {
            if (tn == 1) return launch_mask<1, true, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
            if (tn == 3) return launch_mask<3, true, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
            return launch_mask<5, true, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
        }
        if (tn == 1) return launch_mask<1, false, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
        if (tn == 3) return launch_mask<3, false, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
        return launch_mask<5, false, VT>(f, a, ub, ue, l0, l1, maxu, persistent, s);
    };
    const int nl = int(f->unit_off.size()) - 1;
    const std::vector<int64_t>& bo = f->boff[wpb_slot(f->wpb)];
    int v = 0;
    while (v < nl) {
        const int64_t cnt_v = f->unit_off[v + 1] - f->unit_off[v];  // 64-entry units: the grouping criterion
        if (cnt_v > f->persist_max) {
            kc_status st = go(bo[v], bo[v + 1], v, v + 1, bo[v + 1] - bo[v], false);
            if (st == KC_OK) st = after(v, v + 1);
            if (st != KC_OK) return st;
            ++v;
            continue;
        }
        int w = v;
        int64_t maxb = 0;
        while (w < nl && f->unit_off[w + 1] - f->unit_off[w] <= f->persist_max) {
            maxb = std::max<int64_t>(maxb, bo[w + 1] - bo[w]);
            ++w;
        }
        kc_status st = maxb > 0 ? go(0, 0, v, w, maxb, true) : KC_OK;  // a run of empty levels needs nothing
        if (st == KC_OK) st = after(v, w);
        if (st != KC_OK) return st;
        v = w;
    }
    return KC_OK;
}

// The factorization by supernodal groups: one launch per level of the group DAG.
template <int TN>
kc_status launch_groups_tn(const kc_factor* f, const IcholArgs<float>& a, hipStream_t s) {
    const size_t lds = (size_t(f->cap) + 1) * sizeof(int32_t);
    const size_t nl = f->goff.size() - 1;
    for (size_t v = 0; v < nl; ++v) {
        const int64_t ub = f->goff[v], ue = f->goff[v + 1];
        if (ue <= ub) continue;
        ichol_group<TN><<<unsigned(ue - ub), kWave, lds, s>>>(a, f->groups, f->gunits, ub, ue);
        KC_LAUNCH_CHECK();
    }
    return KC_OK;
}

kc_status launch_groups(const kc_factor* f, int tn, double ell, int pol, double tau, hipStream_t s) {
    const IcholArgs<float> a = ichol_args<float>(f, ell, nullptr, pol, tau);
    if (tn == 1) return launch_groups_tn<1>(f, a, s);
    if (tn == 3) return launch_groups_tn<3>(f, a, s);
    return launch_groups_tn<5>(f, a, s);
}

// Whether a factorization of f runs by supernodal groups (not for update counting).
bool groups_on(const kc_factor* f, bool count) {
    return f->use_groups && f->groups && !count && f->prec == KC_MIXED && f->max_row <= f->stage_max;
}

// Forward sweep of levels [l0, l1): y = L^-1 P b for right-hand sides r0 .. r0+NR-1.
template <typename VT, int NR>
kc_status fwd_levels(const kc_factor* f, const double* b, int ld, int r0, double* y, size_t l0, size_t l1,
                     hipStream_t s) {
    const VT* Lv = static_cast<const VT*>(f->L);
    for (size_t v = l0; v < l1; ++v) {
        const int64_t rb = f->fwd_off[v], re = f->fwd_off[v + 1];
        if (re <= rb) continue;
        if (re - rb >= kWideRows)
            fwd_wide<VT, NR><<<grid_for(re - rb, kWavesPerBlock), kBlock, 0, s>>>(
                f->fwd_rows, rb, re, f->rowptr, f->rowend, f->colidx, Lv, f->diag, f->perm, b, ld, r0, y);
        else
            fwd_solve<VT, NR><<<grid_for(re - rb, kWavesPerBlock), kBlock, 0, s>>>(
                f->fwd_rows, rb, re, f->rowptr, f->rowend, f->colidx, Lv, f->diag, f->perm, b, ld, r0, y);
        KC_LAUNCH_CHECK();
    }
    return KC_OK;
}

// Backward sweep: x = P^T L^-T y for right-hand sides r0 .. r0+NR-1.
template <typename VT, int NR>
kc_status bwd_levels(const kc_factor* f, double* x, int ld, int r0, double* y, double* partial, hipStream_t s) {
    const VT* Lc = static_cast<const VT*>(f->Lcsc);
    const size_t nr = f->short_off.size() - 1;
    for (size_t v = 0; v < nr; ++v) {
        const int64_t sb = f->short_off[v], se = f->short_off[v + 1];
        if (se > sb) {
            bwd_solve<VT, NR><<<grid_for(se - sb, kWavesPerBlock), kBlock, 0, s>>>(
                f->bwd_short, sb, se, f->colptr, f->rowidx, Lc, f->diag, f->perm, ld, r0, y, x);
            KC_LAUNCH_CHECK();
        }
    }
    if (f->top_off.empty()) return KC_OK;
    if (f->nfine > 0) {
        bwd_partial<VT, NR><<<grid_for(f->nfine, kWavesPerBlock), kBlock, 0, s>>>(
            f->bwd_chunks, 0, f->nfine, f->colptr, f->rowidx, Lc, ld, r0, y, partial);
        KC_LAUNCH_CHECK();
    }
    const size_t nt = f->top_off.size() - 1;
    for (size_t v = 0; v < nt; ++v) {
        const int64_t cb = f->nfine + f->tchunk_off[v], ce = f->nfine + f->tchunk_off[v + 1];
        if (ce > cb) {
            bwd_partial<VT, NR><<<grid_for(ce - cb, kWavesPerBlock), kBlock, 0, s>>>(
                f->bwd_chunks, cb, ce, f->colptr, f->rowidx, Lc, ld, r0, y, partial);
            KC_LAUNCH_CHECK();
        }
        const int64_t tb = f->top_off[v], te = f->top_off[v + 1];
        if (te > tb) {
            bwd_finish<VT, NR><<<unsigned(te - tb), kBlock, 0, s>>>(
                f->bwd_top, tb, te, f->colptr, f->rowidx, Lc, f->diag, f->perm, ld, r0, partial, y, x);
            KC_LAUNCH_CHECK();
        }
    }
    return KC_OK;
}

// Calls fn(std::integral_constant<int, NR>(), r0) for each pass of at most
// kMaxRhsPerPass right-hand sides, NR being the pass's width.
template <typename Fn>
kc_status for_passes(int nrhs, Fn fn) {
    for (int r0 = 0; r0 < nrhs; r0 += kMaxRhsPerPass) {
        const int nr = std::min(kMaxRhsPerPass, nrhs - r0);
        kc_status st;
        switch (nr) {
            case 1: st = fn(std::integral_constant<int, 1>(), r0); break;
            case 2: st = fn(std::integral_constant<int, 2>(), r0); break;
            case 3: st = fn(std::integral_constant<int, 3>(), r0); break;
            case 4: st = fn(std::integral_constant<int, 4>(), r0); break;
            case 5: st = fn(std::integral_constant<int, 5>(), r0); break;
            case 6: st = fn(std::integral_constant<int, 6>(), r0); break;
            case 7: st = fn(std::integral_constant<int, 7>(), r0); break;
            default: st = fn(std::integral_constant<int, 8>(), r0); break;
        }
        if (st != KC_OK) return st;
    }
    return KC_OK;
}

template <typename VT>
kc_status solve_typed(const kc_factor* f, const double* b, double* x, int nrhs, double* y, double* partial,
                      hipStream_t s) {
    const size_t nl = f->fwd_off.size() - 1;
    return for_passes(nrhs, [&](auto w, int r0) {
        constexpr int NR = decltype(w)::value;
        const kc_status st = fwd_levels<VT, NR>(f, b, nrhs, r0, y, 0, nl, s);
        return st != KC_OK ? st : bwd_levels<VT, NR>(f, x, nrhs, r0, y, partial, s);
    });
}

// Factorization and solve with the forward sweep overlapped: once the launch
// covering factor levels [l0, l1) is enqueued on s, an event recorded after it
// lets the second stream `aux` run the forward sweep of the same levels while s
// goes on with the next factor levels.  A row of level v reads only L entries of
// columns at levels <= v and y of rows at levels < v, and no later factor level
// writes them, so the two streams never touch the same data out of order.  The
// backward sweep needs the whole factor and runs on s after both.
template <typename VT>
kc_status factorize_solve_typed(kc_factor* f, int tn, double ell, const double* ells, int pol, double tau,
                                const double* b, double* x, int nrhs, double* y, double* partial, hipStream_t s) {
    hipStream_t aux = f->aux;
    hipEvent_t ev = f->aux_ev;
    auto after = [&](int l0, int l1) -> kc_status {
        KC_HIP(hipEventRecord(ev, s));
        KC_HIP(hipStreamWaitEvent(aux, ev, 0));
        return for_passes(nrhs, [&](auto w, int r0) {
            constexpr int NR = decltype(w)::value;
            return fwd_levels<VT, NR>(f, b, nrhs, r0, y, size_t(l0), size_t(l1), aux);
        });
    };
    kc_status st = launch_levels<VT>(f, tn, false, ell, ells, pol, tau, s, after);
    // whatever was enqueued on aux must finish before s goes on, also after an error
    KC_HIP(hipEventRecord(ev, aux));
    KC_HIP(hipStreamWaitEvent(s, ev, 0));
    if (st != KC_OK) return st;
    return for_passes(nrhs, [&](auto w, int r0) {
        constexpr int NR = decltype(w)::value;
        return bwd_levels<VT, NR>(f, x, nrhs, r0, y, partial, s);
    });
}

size_t solve_scratch_bytes(const kc_factor* f, int32_t nrhs) {
    return align256(size_t(f->n) * size_t(nrhs) * sizeof(double)) +
           size_t(std::max<int64_t>(f->max_slots, 1)) * kMaxRhsPerPass * sizeof(double);
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
        case KC_ERANGE: return "problem too large for the index types";
    }
    return "unknown status";
}

const char* kc_last_error(void) { return kc::g_err.c_str(); }

int32_t kc_device_count(void) {
    int c = 0;
    if (hipGetDeviceCount(&c) != hipSuccess) return 0;
    return c;
}

static kc_status check_points(const double* x, int64_t n, int32_t d, double rho, kc_rule rule) {
    if (!x || n < 1 || d < 1 || !(rho > 0.0) || !std::isfinite(rho) || (rule != KC_RULE_MAX && rule != KC_RULE_MIN)) {
        kc::set_error("kc_analyze: need x != NULL, n >= 1, d >= 1, finite rho > 0, rule MAX or MIN");
        return KC_EINVAL;
    }
    if (n >= (int64_t(1) << 31) - 1) {
        kc::set_error("kc_analyze: n must be below 2^31 - 1");
        return KC_ERANGE;
    }
    for (int64_t i = 0; i < n * d; ++i)
        if (!std::isfinite(x[i])) {
            kc::set_error("kc_analyze: non-finite coordinate");
            return KC_EINVAL;
        }
    return KC_OK;
}

static void analyze_one(const double* x, int64_t n, int32_t d, double rho, kc_rule rule, int32_t nthreads,
                        kc::Plan& p, bool supernodal = false) {
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
    if (supernodal && p.nnz() < (int64_t(1) << 32) && p.nnz_rows() < (int64_t(1) << 32))
        kc::supernodal_transform(p, nthreads);
    auto t2 = std::chrono::steady_clock::now();
    if (p.nnz() < (int64_t(1) << 32) && p.nnz_rows() < (int64_t(1) << 32)) kc::build_schedule(p, nthreads);
    auto t3 = std::chrono::steady_clock::now();
    p.t_order = std::chrono::duration<double>(t1 - t0).count();
    p.t_pattern = std::chrono::duration<double>(t2 - t1).count();
    p.t_schedule = std::chrono::duration<double>(t3 - t2).count();
}

kc_status kc_analyze(const double* x, int64_t n, int32_t d, double rho, kc_rule rule, int32_t nthreads,
                     kc_plan** out) {
    if (!out) {
        kc::set_error("kc_analyze: out is NULL");
        return KC_EINVAL;
    }
    *out = nullptr;
    const kc_status st = check_points(x, n, d, rho, rule);
    if (st != KC_OK) return st;
    kc_plan* plan = new (std::nothrow) kc_plan;
    if (!plan) return KC_ENOMEM;
    try {
        analyze_one(x, n, d, rho, rule, nthreads, plan->p);
    } catch (const std::bad_alloc&) {
        delete plan;
        kc::set_error("kc_analyze: out of host memory");
        return KC_ENOMEM;
    }
    if (plan->p.nnz() >= (int64_t(1) << 32) || plan->p.nnz_rows() >= (int64_t(1) << 32)) {
        delete plan;
        kc::set_error("kc_analyze: nnz(S) >= 2^32");
        return KC_ERANGE;
    }
    *out = plan;
    return KC_OK;
}

kc_status kc_analyze_supernodal(const double* x, int64_t n, int32_t d, double rho, int32_t nthreads,
                                kc_plan** out) {
    if (!out) return KC_EINVAL;
    *out = nullptr;
    const kc_status st = check_points(x, n, d, rho, KC_RULE_MAX);
    if (st != KC_OK) return st;
    kc_plan* plan = new (std::nothrow) kc_plan;
    if (!plan) return KC_ENOMEM;
    try {
        analyze_one(x, n, d, rho, KC_RULE_MAX, nthreads, plan->p, true);
    } catch (const std::bad_alloc&) {
        delete plan;
        kc::set_error("kc_analyze_supernodal: out of host memory");
        return KC_ENOMEM;
    }
    if (plan->p.nnz() >= (int64_t(1) << 32) || plan->p.nnz_rows() >= (int64_t(1) << 32)) {
        delete plan;
        kc::set_error("kc_analyze_supernodal: nnz(S) >= 2^32");
        return KC_ERANGE;
    }
    *out = plan;
    return KC_OK;
}

kc_status kc_plan_supernodes(const kc_plan* plan, int64_t* snode_ptr, int64_t* nsuper) {
    if (!plan || !nsuper) return KC_EINVAL;
    const kc::Plan& p = plan->p;
    if (p.snode_ptr.empty()) {
        *nsuper = 0;
        return KC_OK;
    }
    *nsuper = int64_t(p.snode_ptr.size()) - 1;
    if (snode_ptr) std::memcpy(snode_ptr, p.snode_ptr.data(), p.snode_ptr.size() * sizeof(int64_t));
    return KC_OK;
}

kc_status kc_analyze_batched(const double* x, const int64_t* counts, int32_t ninst, int32_t d, double rho,
                             kc_rule rule, int32_t nthreads, kc_plan** out) {
    if (!out) return KC_EINVAL;
    *out = nullptr;
    if (!counts || ninst < 1) {
        kc::set_error("kc_analyze_batched: need counts and ninst >= 1");
        return KC_EINVAL;
    }
    std::vector<int64_t> off(size_t(ninst) + 1, 0);
    for (int32_t i = 0; i < ninst; ++i) {
        if (counts[i] < 1) {
            kc::set_error("kc_analyze_batched: every instance needs at least one point");
            return KC_EINVAL;
        }
        off[i + 1] = off[i] + counts[i];
    }
    const kc_status st = check_points(x, off[ninst], d, rho, rule);
    if (st != KC_OK) return st;
    kc_plan* plan = new (std::nothrow) kc_plan;
    if (!plan) return KC_ENOMEM;
    try {
        std::vector<kc::Plan> parts(static_cast<size_t>(ninst));
        int nt = nthreads > 0 ? nthreads : int(std::max(1u, std::thread::hardware_concurrency()));
        nt = std::min(nt, ninst);
        std::atomic<int32_t> next{0};
        auto work = [&]() {
            for (;;) {
                const int32_t i = next.fetch_add(1);
                if (i >= ninst) break;
                analyze_one(x + size_t(off[i]) * d, counts[i], d, rho, rule, 1, parts[size_t(i)]);
            }
        };
        std::vector<std::thread> pool;
        for (int t = 1; t < nt; ++t) pool.emplace_back(work);
        work();
        for (auto& th : pool) th.join();
        kc::merge_plans(parts, plan->p);
    } catch (const std::bad_alloc&) {
        delete plan;
        kc::set_error("kc_analyze_batched: out of host memory");
        return KC_ENOMEM;
    }
    if (plan->p.nnz() >= (int64_t(1) << 32) || plan->p.nnz_rows() >= (int64_t(1) << 32)) {
        delete plan;
        kc::set_error("kc_analyze_batched: nnz(S) of the batch >= 2^32");
        return KC_ERANGE;
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
    info->ninst = p.ninst;
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

kc_status kc_plan_set_delta_limit(kc_plan* plan, uint32_t delta_limit, int64_t* nescapes) {
    if (!plan || delta_limit < 1 || delta_limit > 65536) {
        kc::set_error("kc_plan_set_delta_limit: need a plan and 1 <= delta_limit <= 65536");
        return KC_EINVAL;
    }
    try {
        plan->p.delta_limit = delta_limit;
        kc::encode_row_deltas(plan->p, 0);
    } catch (const std::bad_alloc&) {
        kc::set_error("kc_plan_set_delta_limit: out of host memory");
        return KC_ENOMEM;
    }
    if (nescapes) *nescapes = int64_t(plan->p.esc.size());
    return KC_OK;
}

void kc_plan_destroy(kc_plan* plan) { delete plan; }

kc_status kc_factor_bytes(const kc_plan* plan, kc_prec prec, size_t* bytes) {
    if (!plan || !bytes || (prec != KC_FP64 && prec != KC_MIXED)) return KC_EINVAL;
    try {
        *bytes = layout_of(plan->p, backward_schedule(plan->p), prec,
                           prec == KC_MIXED ? group_schedule(plan->p) : GroupSchedule())
                     .total;
    } catch (const std::bad_alloc&) {
        return KC_ENOMEM;
    }
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
    BwdSchedule bs;
    GroupSchedule gs;
    try {
        bs = backward_schedule(p);
        if (prec == KC_MIXED) gs = group_schedule(p);
    } catch (const std::bad_alloc&) {
        return KC_ENOMEM;
    }
    const Layout o = layout_of(p, bs, prec, gs);
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
    const size_t vt = prec == KC_FP64 ? sizeof(double) : sizeof(float);
    f->cap = lds_cap(p);
    f->nbuck = bucket_count(p);
    f->max_row = p.max_row;
    if (factor_lds(f.get(), vt) > kMaxLdsBytes) {
        // rows longer than the LDS holds are read from device memory (row_unstaged)
        const size_t dir = f->nbuck ? size_t(f->nbuck + 1) * sizeof(uint16_t) : 0;
        f->cap = int32_t((kMaxLdsBytes - dir - 16) / (vt + sizeof(int32_t)) / 16 * 16);
    }
    f->stage_max = f->cap - 2;
    {
        // a workgroup covers 64 * wpb entries of one column: more wavefronts share one
        // staged row on long columns, fewer leave less padding on short ones
        const double avg = double(p.nnz()) / double(std::max<int64_t>(1, p.n));
        f->wpb = avg >= 1024.0 ? 4 : avg >= 512.0 ? 2 : 1;
    }
    char* base = static_cast<char*>(ws_dev);
    f->n = p.n;
    f->nnz = p.nnz();
    f->nnz_rows = p.nnz_rows();
    f->d = p.d;
    f->prec = prec;
    f->nunits = int64_t(p.units.size());
    {
        int dev = 0;
        KC_HIP(hipGetDevice(&dev));
        KC_HIP(hipDeviceGetAttribute(&f->num_cu, hipDeviceAttributeMultiprocessorCount, dev));
    }
    f->counters = reinterpret_cast<unsigned long long*>(base + o.counters);
    f->xh = reinterpret_cast<double*>(base + o.xh);
    f->perm = reinterpret_cast<int32_t*>(base + o.perm);
    f->colptr = reinterpret_cast<int64_t*>(base + o.colptr);
    f->rowidx = reinterpret_cast<int32_t*>(base + o.rowidx);
    f->csc2csr = reinterpret_cast<uint32_t*>(base + o.csc2csr);
    f->rowptr = reinterpret_cast<int64_t*>(base + o.rowptr);
    f->rowend = reinterpret_cast<int64_t*>(base + o.rowend);
    f->colidx = reinterpret_cast<int32_t*>(base + o.colidx);
    f->cdelta = reinterpret_cast<uint32_t*>(base + o.cdelta);
    f->escptr = reinterpret_cast<uint32_t*>(base + o.escptr);
    f->esc = reinterpret_cast<int32_t*>(base + o.esc);
    f->L = base + o.L;
    f->Lcsc = base + o.Lcsc;
    f->diag = prec == KC_MIXED ? reinterpret_cast<double*>(base + o.diag) : nullptr;
    f->units = reinterpret_cast<Unit*>(base + o.units);
    f->unit_off_dev = reinterpret_cast<int64_t*>(base + o.unit_off);
    for (int w = 0; w < 3; ++w) {
        for (int r = 0; r < 2; ++r) f->bunits[r][w] = reinterpret_cast<Unit*>(base + o.bunits[r][w]);
        f->bunits_alt[w] = f->bunits[KC_ORDER_LONGEST][w];
        f->boff_dev[w] = reinterpret_cast<int64_t*>(base + o.boff[w]);
    }
    f->fwd_rows = reinterpret_cast<int32_t*>(base + o.fwd);
    f->bwd_short = reinterpret_cast<int32_t*>(base + o.bshort);
    f->bwd_top = reinterpret_cast<kc::TopCol*>(base + o.blong);
    f->bwd_chunks = reinterpret_cast<kc::BwdChunk*>(base + o.bchunks);
    f->inst = p.ninst > 1 ? reinterpret_cast<int32_t*>(base + o.inst) : nullptr;
    f->ninst = p.ninst;
    f->unit_off = p.unit_off;
    f->fwd_off = p.fwd_off;
    f->short_off = bs.short_off;
    f->top_off = bs.top_off;
    f->tchunk_off = bs.tchunk_off;
    f->nfine = bs.nfine;
    f->max_slots = bs.max_slots;

    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t n = size_t(p.n), nnz = size_t(p.nnz()), nnzr = size_t(p.nnz_rows());
    KC_HIP(hipMemcpyAsync(f->perm, p.perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->colptr, p.colptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->rowidx, p.rowidx.data(), nnz * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->csc2csr, p.csc2csr.data(), nnz * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->rowptr, p.rowptr.data(), (n + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->rowend, p.rowend.data(), n * sizeof(int64_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->colidx, p.colidx.data(), nnzr * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->cdelta, p.cdelta.data(), nnzr * sizeof(uint16_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->escptr, p.escptr.data(), (size_t(p.n) + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    if (!p.esc.empty())
        KC_HIP(hipMemcpyAsync(f->esc, p.esc.data(), p.esc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->units, p.units.data(), p.units.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
    KC_HIP(hipMemcpyAsync(f->unit_off_dev, p.unit_off.data(), p.unit_off.size() * sizeof(int64_t),
                          hipMemcpyHostToDevice, s));
    // both unit orders, unless no level exceeds what the device holds at once
    // (then the order cannot matter, and LONGEST shares SPATIAL's arrays)
    f->order = default_order(p, f->num_cu);
    const bool both = order_matters(p, f->num_cu);
    std::vector<int32_t> walk;
    try {
        if (both) walk = unit_walks(p);
    } catch (const std::bad_alloc&) {
        return KC_ENOMEM;
    }
    for (int w = 0; w < 3; ++w) {
        for (int r = 0; r < (both ? 2 : 1); ++r) {
            std::vector<Unit> bu;
            try {
                block_units(p.units, p.unit_off, big_plan(p), 1 << w, r, walk, bu, f->boff[w]);
            } catch (const std::bad_alloc&) {
                return KC_ENOMEM;
            }
            if (!bu.empty())
                KC_HIP(hipMemcpyAsync(f->bunits[r][w], bu.data(), bu.size() * sizeof(Unit), hipMemcpyHostToDevice, s));
            KC_HIP(hipStreamSynchronize(s));  // bu is a local buffer
        }
        if (!both) f->bunits[KC_ORDER_LONGEST][w] = f->bunits[KC_ORDER_SPATIAL][w];
        KC_HIP(hipMemcpyAsync(f->boff_dev[w], f->boff[w].data(), f->boff[w].size() * sizeof(int64_t),
                              hipMemcpyHostToDevice, s));
    }
    KC_HIP(hipMemcpyAsync(f->fwd_rows, p.fwd_rows.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!bs.shortc.empty())
        KC_HIP(hipMemcpyAsync(f->bwd_short, bs.shortc.data(), bs.shortc.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, s));
    if (!bs.topc.empty())
        KC_HIP(hipMemcpyAsync(f->bwd_top, bs.topc.data(), bs.topc.size() * sizeof(kc::TopCol),
                              hipMemcpyHostToDevice, s));
    if (!bs.chunks.empty())
        KC_HIP(hipMemcpyAsync(f->bwd_chunks, bs.chunks.data(), bs.chunks.size() * sizeof(kc::BwdChunk),
                              hipMemcpyHostToDevice, s));
    if (f->inst) KC_HIP(hipMemcpyAsync(f->inst, p.inst.data(), n * sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (!gs.groups.empty()) {  // a supernodal plan in mixed precision: groups on the matrix cores by default
        f->groups = reinterpret_cast<kc::GroupDesc*>(base + o.groups);
        f->gunits = reinterpret_cast<int2*>(base + o.gunits);
        f->goff = gs.off;
        f->use_groups = true;
        KC_HIP(hipMemcpyAsync(f->groups, gs.groups.data(), gs.groups.size() * sizeof(kc::GroupDesc),
                              hipMemcpyHostToDevice, s));
        KC_HIP(hipMemcpyAsync(f->gunits, gs.units.data(), gs.units.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    }
    // the sources are pageable host memory owned by the plan and bs: wait for the copies
    KC_HIP(hipStreamSynchronize(s));
    f->last = s;
    *out = f.release();
    return KC_OK;
}

static kc_status factorize_impl(kc_factor* f, const double* x_dev, double nu, double ell, const double* ells,
                                kc_pivot pivot, double tau, int32_t count_updates, void* stream) {
    const int tn = twonu_of(nu);
    if (!tn) {
        kc::set_error("kc_factorize: nu must be 0.5, 1.5 or 2.5");
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
    const kc_status st = groups_on(f, cnt) ? launch_groups(f, tn, ell, int(pivot), tau, s)
                         : f->prec == KC_FP64 ? launch_levels<double>(f, tn, cnt, ell, ells, int(pivot), tau, s)
                                              : launch_levels<float>(f, tn, cnt, ell, ells, int(pivot), tau, s);
    if (st != KC_OK) return st;
    f->factorized = true;
    f->counted = cnt;
    f->last = s;
    return KC_OK;
}

kc_status kc_factorize(kc_factor* f, const double* x_dev, kc_kernel kernel, kc_pivot pivot, double tau,
                       int32_t count_updates, void* stream) {
    if (!f || !x_dev) return KC_EINVAL;
    if (f->ninst > 1) {
        kc::set_error("kc_factorize: the plan holds a batch; use kc_factorize_batched");
        return KC_EINVAL;
    }
    if (!(kernel.lengthscale > 0.0) || !std::isfinite(kernel.lengthscale)) {
        kc::set_error("kc_factorize: the lengthscale must be finite and positive");
        return KC_EINVAL;
    }
    return factorize_impl(f, x_dev, kernel.nu, kernel.lengthscale, nullptr, pivot, tau, count_updates, stream);
}

kc_status kc_factorize_batched(kc_factor* f, const double* x_dev, double nu, const double* ell_dev, kc_pivot pivot,
                               double tau, int32_t count_updates, void* stream) {
    if (!f || !x_dev || !ell_dev) return KC_EINVAL;
    if (f->ninst < 2) {
        kc::set_error("kc_factorize_batched: the plan holds a single problem; use kc_factorize");
        return KC_EINVAL;
    }
    return factorize_impl(f, x_dev, nu, 0.0, ell_dev, pivot, tau, count_updates, stream);
}

kc_status kc_theta(kc_factor* f, const double* x_dev, kc_kernel kernel, double* theta_dev, void* stream) {
    if (!f || !x_dev || !theta_dev) return KC_EINVAL;
    const int tn = twonu_of(kernel.nu);
    if (!tn || !(kernel.lengthscale > 0.0)) return KC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    zero_u64<<<1, 64, 0, s>>>(f->counters, kNumCounters);
    KC_LAUNCH_CHECK();
    gather_points<<<grid_for(f->n * f->d, kBlock), kBlock, 0, s>>>(x_dev, f->perm, f->n, f->d, f->xh);
    KC_LAUNCH_CHECK();
    if (f->nunits > 0) {
        const dim3 grid(grid_for(f->nunits, kWavesPerBlock));
        const double ell = kernel.lengthscale;
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
    *bytes = solve_scratch_bytes(f, nrhs);
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
    if (scratch_bytes < solve_scratch_bytes(f, nrhs) || reinterpret_cast<uintptr_t>(scratch_dev) % 256) {
        kc::set_error("kc_solve: scratch must be 256-byte aligned and hold kc_solve_bytes bytes");
        return KC_EWORKSPACE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* y = static_cast<double*>(scratch_dev);
    double* partial = reinterpret_cast<double*>(static_cast<char*>(scratch_dev) +
                                                align256(size_t(f->n) * size_t(nrhs) * sizeof(double)));
    const kc_status st = f->prec == KC_FP64 ? solve_typed<double>(f, b_dev, x_dev, nrhs, y, partial, s)
                                            : solve_typed<float>(f, b_dev, x_dev, nrhs, y, partial, s);
    const_cast<kc_factor*>(f)->last = s;
    return st;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Scratch of kc_solve_noalloc: one array per device that loads the library,
// held until the process ends.  In host code `scratch` names a host-side
// stand-in, not device memory: kernels get the address that
// hipGetSymbolAddress returns for the current device (noalloc_scratch).
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(96) << 20;
constexpr int kMaxDevices = 64;
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
kc_status noalloc_scratch(void** out) {
    int dev = 0;
    KC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        kc::set_error("kc_solve_noalloc: device index " + std::to_string(dev) + " beyond the supported range");
        return KC_EINVAL;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        KC_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) {
            kc::set_error("kc_solve_noalloc: hipGetSymbolAddress returned no address for the scratch array");
            return KC_EHIP;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return KC_OK;
}
}  // namespace

extern "C" {

kc_status kc_solve_noalloc(const kc_factor* f, const double* b_dev, double* x_dev, int32_t nrhs, void* stream) {
    if (!f || !b_dev || !x_dev || nrhs < 1) return KC_EINVAL;
    if (b_dev == x_dev) {
        kc::set_error("kc_solve_noalloc: b and x must not alias");
        return KC_EINVAL;
    }
    if (!f->factorized) {
        kc::set_error("kc_solve_noalloc: factor has not been computed");
        return KC_ESTATE;
    }
    const size_t need = solve_scratch_bytes(f, nrhs);
    if (need > kNoAllocScratchBytes) {
        kc::set_error("kc_solve_noalloc: this solve needs " + std::to_string(need) +
                      " bytes of scratch, beyond the library's fixed " + std::to_string(kNoAllocScratchBytes) +
                      "; use kc_solve with caller-owned scratch");
        return KC_EWORKSPACE;
    }
    void* base = nullptr;
    const kc_status got = noalloc_scratch(&base);
    if (got != KC_OK) return got;
    hipStream_t s = static_cast<hipStream_t>(stream);
    double* y = static_cast<double*>(base);
    double* partial = reinterpret_cast<double*>(static_cast<char*>(base) +
                                                align256(size_t(f->n) * size_t(nrhs) * sizeof(double)));
    const kc_status st = f->prec == KC_FP64 ? solve_typed<double>(f, b_dev, x_dev, nrhs, y, partial, s)
                                            : solve_typed<float>(f, b_dev, x_dev, nrhs, y, partial, s);
    const_cast<kc_factor*>(f)->last = s;
    return st;
}

kc_status kc_factorize_solve(kc_factor* f, const double* x_dev, kc_kernel kernel, const double* ell_dev,
                             kc_pivot pivot, double tau, const double* b_dev, double* x_out, int32_t nrhs,
                             void* scratch_dev, size_t scratch_bytes, void* stream) {
    if (!f || !x_dev || !b_dev || !x_out || !scratch_dev || nrhs < 1) return KC_EINVAL;
    if ((f->ninst > 1) != (ell_dev != nullptr)) {
        kc::set_error("kc_factorize_solve: pass ell_dev exactly for batch plans");
        return KC_EINVAL;
    }
    if (b_dev == x_out) {
        kc::set_error("kc_factorize_solve: b and x must not alias");
        return KC_EINVAL;
    }
    const int tn = twonu_of(kernel.nu);
    if (!tn || (!ell_dev && (!(kernel.lengthscale > 0.0) || !std::isfinite(kernel.lengthscale)))) {
        kc::set_error("kc_factorize_solve: nu must be 0.5, 1.5 or 2.5 and the lengthscale finite and positive");
        return KC_EINVAL;
    }
    if (pivot != KC_PIVOT_ZERO && pivot != KC_PIVOT_SHIFT) return KC_EINVAL;
    if (pivot == KC_PIVOT_SHIFT && !(tau > 0.0 && std::isfinite(tau))) {
        kc::set_error("kc_factorize_solve: KC_PIVOT_SHIFT needs a finite tau > 0");
        return KC_EINVAL;
    }
    if (scratch_bytes < solve_scratch_bytes(f, nrhs) || reinterpret_cast<uintptr_t>(scratch_dev) % 256) {
        kc::set_error("kc_factorize_solve: scratch must be 256-byte aligned and hold kc_solve_bytes bytes");
        return KC_EWORKSPACE;
    }
    if (!f->aux) {  // the second stream, default priority, on the current device
        KC_HIP(hipStreamCreateWithFlags(&f->aux, hipStreamNonBlocking));
        if (hipEventCreateWithFlags(&f->aux_ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(f->aux);
            f->aux = nullptr;
            kc::set_error("kc_factorize_solve: hipEventCreateWithFlags failed");
            return KC_EHIP;
        }
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    zero_u64<<<1, 64, 0, s>>>(f->counters, kNumCounters);
    KC_LAUNCH_CHECK();
    gather_points<<<grid_for(f->n * f->d, kBlock), kBlock, 0, s>>>(x_dev, f->perm, f->n, f->d, f->xh);
    KC_LAUNCH_CHECK();
    double* y = static_cast<double*>(scratch_dev);
    double* partial = reinterpret_cast<double*>(static_cast<char*>(scratch_dev) +
                                                align256(size_t(f->n) * size_t(nrhs) * sizeof(double)));
    const double ell = ell_dev ? 0.0 : kernel.lengthscale;
    kc_status st;
    if (groups_on(f, false)) {  // the group DAG has its own levels: factor, then both sweeps
        st = launch_groups(f, tn, ell, int(pivot), tau, s);
        if (st == KC_OK) st = solve_typed<float>(f, b_dev, x_out, nrhs, y, partial, s);
    } else {
        st = f->prec == KC_FP64
                 ? factorize_solve_typed<double>(f, tn, ell, ell_dev, int(pivot), tau, b_dev, x_out, nrhs, y, partial, s)
                 : factorize_solve_typed<float>(f, tn, ell, ell_dev, int(pivot), tau, b_dev, x_out, nrhs, y, partial, s);
    }
    if (st != KC_OK) return st;
    f->factorized = true;
    f->counted = false;
    f->last = s;
    return KC_OK;
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
    st->nonfinite = int64_t(c[kNonfinite]);
    st->match_errors = int64_t(c[kMatchErr]);
    return KC_OK;
}

}  // extern "C"

namespace {
uint64_t match_blocks(const kc_factor* f) { return uint64_t((f->nunits + kWavesPerBlock - 1) / kWavesPerBlock); }

size_t match_bytes_of(const kc_factor* f) {
    return align256(size_t(f->nnz) * sizeof(uint64_t)) +
           align256(size_t(std::max<uint64_t>(match_blocks(f), 1)) * sizeof(uint64_t)) +
           size_t(f->match_words) * sizeof(uint64_t);
}

// Reads one counter back (synchronous on s).
kc_status read_counter(const kc_factor* f, int which, hipStream_t s, unsigned long long* out) {
    KC_HIP(hipMemcpyAsync(out, f->counters + which, sizeof(*out), hipMemcpyDeviceToHost, s));
    KC_HIP(hipStreamSynchronize(s));
    return KC_OK;
}
}  // namespace

extern "C" {

kc_status kc_factor_match_bytes(kc_factor* f, void* stream, size_t* bytes) {
    if (!f || !bytes) return KC_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!f->match_counted) {
        unsigned long long total = 0;
        if (f->nunits > 0) {
            zero_u64<<<1, 64, 0, s>>>(f->counters + kMatchTotal, 1);
            KC_LAUNCH_CHECK();
            const unsigned g = unsigned(std::min<int64_t>(grid_for(f->nunits, kWavesPerBlock), 4096));
            match_total_kernel<<<g, kBlock, 0, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->csc2csr, f->rowptr,
                                                    f->rowend, f->counters);
            KC_LAUNCH_CHECK();
            const kc_status st = read_counter(f, kMatchTotal, s, &total);
            if (st != KC_OK) return st;
        }
        f->match_words = total;
        f->match_counted = true;
    }
    *bytes = match_bytes_of(f);
    return KC_OK;
}

kc_status kc_factor_match_build(kc_factor* f, void* buf_dev, size_t bytes, void* stream) {
    if (!f) return KC_EINVAL;
    if (!buf_dev) {  // detach: back to the index merge
        f->mmeta = nullptr;
        f->mwords = nullptr;
        f->mwords_n = 0;
        return KC_OK;
    }
    size_t need = 0;
    kc_status st = kc_factor_match_bytes(f, stream, &need);
    if (st != KC_OK) return st;
    if (bytes < need || reinterpret_cast<uintptr_t>(buf_dev) % 256) {
        kc::set_error("kc_factor_match_build: the buffer must be 256-byte aligned and hold kc_factor_match_bytes (" +
                      std::to_string(need) + ") bytes");
        return KC_EWORKSPACE;
    }
    const size_t lds = size_t(kWavesPerBlock) * size_t(f->cap) * sizeof(int32_t);
    if (lds > kMaxLdsBytes || f->max_row > f->stage_max) {
        kc::set_error("kc_factor_match_build: a row of S is too long to stage for the mask build");
        return KC_ERANGE;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* base = static_cast<char*>(buf_dev);
    const uint64_t nb = match_blocks(f);
    uint64_t* meta = reinterpret_cast<uint64_t*>(base);
    uint64_t* bsum = reinterpret_cast<uint64_t*>(base + align256(size_t(f->nnz) * sizeof(uint64_t)));
    uint64_t* words = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(bsum) +
                                                  align256(size_t(std::max<uint64_t>(nb, 1)) * sizeof(uint64_t)));
    const uint64_t W = f->match_words;
    f->mmeta = nullptr;  // the index merge until the masks are complete
    f->mwords = nullptr;
    f->mwords_n = 0;
    if (f->nunits > 0) {
        match_count_kernel<<<unsigned(nb), kBlock, 0, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->csc2csr,
                                                          f->rowptr, f->rowend, meta, bsum);
        KC_LAUNCH_CHECK();
        std::vector<uint64_t> h;
        try {
            h.resize(size_t(nb));
        } catch (const std::bad_alloc&) {
            return KC_ENOMEM;
        }
        KC_HIP(hipMemcpyAsync(h.data(), bsum, size_t(nb) * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
        KC_HIP(hipStreamSynchronize(s));
        uint64_t run = 0;
        for (uint64_t b = 0; b < nb; ++b) {
            const uint64_t t = h[size_t(b)];
            h[size_t(b)] = run;
            run += t;
        }
        if (run != W) {
            kc::set_error("kc_factor_match_build: mask word counts disagree (" + std::to_string(run) + " vs " +
                          std::to_string(W) + ")");
            return KC_ESTATE;
        }
        KC_HIP(hipMemcpyAsync(bsum, h.data(), size_t(nb) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        KC_HIP(hipStreamSynchronize(s));  // h is a local buffer
        match_base_kernel<<<unsigned(nb), kBlock, 0, s>>>(f->units, f->nunits, f->colptr, bsum, meta);
        KC_LAUNCH_CHECK();
        if (W > 0) {
            fill_u64<<<unsigned(std::min<uint64_t>((W + kBlock - 1) / kBlock, 16384)), kBlock, 0, s>>>(words, W, 0);
            KC_LAUNCH_CHECK();
        }
        zero_u64<<<1, 64, 0, s>>>(f->counters + kMatchErr, 1);
        KC_LAUNCH_CHECK();
        match_masks_kernel<<<unsigned(nb), kBlock, lds, s>>>(f->units, f->nunits, f->colptr, f->rowidx, f->csc2csr,
                                                            f->rowptr, f->rowend, f->colidx, f->cap, meta, words, W,
                                                            f->counters);
        KC_LAUNCH_CHECK();
        unsigned long long errs = 0;
        st = read_counter(f, kMatchErr, s, &errs);
        if (st != KC_OK) return st;
        if (errs) {
            kc::set_error("kc_factor_match_build: " + std::to_string(errs) + " entries fell outside the mask buffer");
            return KC_ESTATE;
        }
    }
    f->mmeta = meta;
    f->mwords = words;
    f->mwords_n = W;
    f->last = s;
    return KC_OK;
}

kc_status kc_factor_export_L(const kc_factor* f, double* vals) {
    if (!f || !vals) return KC_EINVAL;
    if (!f->factorized) return KC_ESTATE;
    KC_HIP(hipStreamSynchronize(f->last));
    const size_t nnz = size_t(f->nnz);
    if (f->prec == KC_FP64) {
        KC_HIP(hipMemcpy(vals, f->Lcsc, nnz * sizeof(double), hipMemcpyDeviceToHost));
    } else {
        std::vector<float> v(nnz);
        std::vector<double> dg(size_t(f->n));
        std::vector<int64_t> colptr(size_t(f->n) + 1);
        KC_HIP(hipMemcpy(v.data(), f->Lcsc, nnz * sizeof(float), hipMemcpyDeviceToHost));
        KC_HIP(hipMemcpy(dg.data(), f->diag, dg.size() * sizeof(double), hipMemcpyDeviceToHost));
        KC_HIP(hipMemcpy(colptr.data(), f->colptr, colptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
        for (size_t e = 0; e < nnz; ++e) vals[e] = double(v[e]);
        for (int64_t j = 0; j < f->n; ++j) vals[colptr[size_t(j)]] = dg[size_t(j)];
    }
    return KC_OK;
}

void kc_factor_destroy(kc_factor* f) {
    if (!f) return;
    if (f->aux_ev) (void)hipEventDestroy(f->aux_ev);
    if (f->aux) (void)hipStreamDestroy(f->aux);
    delete f;
}

kc_status kc_factor_tune(kc_factor* f, const double* x_dev, double nu, double ell, const double* ell_dev,
                         kc_pivot pivot, double tau, int32_t reps, void* stream, int32_t* chosen_wpb) {
    if (!f || !x_dev || reps < 1) return KC_EINVAL;
    if ((f->ninst > 1) != (ell_dev != nullptr)) {
        kc::set_error("kc_factor_tune: pass ell_dev exactly for batch plans");
        return KC_EINVAL;
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    const size_t vt = f->prec == KC_FP64 ? sizeof(double) : sizeof(float);
    hipEvent_t a = nullptr, b = nullptr;
    KC_HIP(hipEventCreate(&a));
    KC_HIP(hipEventCreate(&b));
    int best = f->wpb;
    int64_t best_pm = f->persist_max;
    int32_t best_order = f->order;
    float best_ms = 1e30f;
    // level grouping: levels with at most `pm` units share persistent launches
    const int64_t kGroupings[] = {0, 256, 4096, INT64_MAX};
    for (int wpb : {1, 2, 4}) {
        if (factor_lds(f, vt) > kMaxLdsBytes) continue;
        for (int64_t pm : kGroupings) for (int32_t order : {KC_ORDER_SPATIAL, KC_ORDER_LONGEST}) {
            // no level exceeds what the device holds at once: both orders share one array
            if (order == KC_ORDER_LONGEST && f->bunits[KC_ORDER_LONGEST][0] == f->bunits[KC_ORDER_SPATIAL][0])
                continue;
            f->wpb = wpb;
            f->persist_max = pm;
            f->order = order;
            kc_status st = factorize_impl(f, x_dev, nu, ell, ell_dev, pivot, tau, 0, stream);  // warm-up
            if (st != KC_OK) {
                // e.g. a persistent launch that does not fit: skip this grouping
                (void)hipGetLastError();
                (void)hipStreamSynchronize(s);
                continue;
            }
            KC_HIP(hipEventRecord(a, s));
            for (int r = 0; r < reps && st == KC_OK; ++r)
                st = factorize_impl(f, x_dev, nu, ell, ell_dev, pivot, tau, 0, stream);
            KC_HIP(hipEventRecord(b, s));
            KC_HIP(hipEventSynchronize(b));
            if (st != KC_OK) continue;
            float ms = 0.f;
            KC_HIP(hipEventElapsedTime(&ms, a, b));
            if (ms < best_ms) {
                best_ms = ms;
                best = wpb;
                best_pm = pm;
                best_order = order;
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    f->wpb = best;
    f->persist_max = best_pm;
    f->order = best_order;
    if (chosen_wpb) *chosen_wpb = best;
    return KC_OK;
}

kc_status kc_factor_set_schedule(kc_factor* f, int32_t wpb, int64_t persist_max, kc_unit_order order) {
    if (!f || (wpb != 1 && wpb != 2 && wpb != 4) || persist_max < 0 ||
        (order != KC_ORDER_SPATIAL && order != KC_ORDER_LONGEST)) {
        kc::set_error("kc_factor_set_schedule: wavefronts per block must be 1, 2 or 4, persist_max >= 0 and "
                      "order SPATIAL or LONGEST");
        return KC_EINVAL;
    }
    const size_t vt = f->prec == KC_FP64 ? sizeof(double) : sizeof(float);
    if (factor_lds(f, vt) > kMaxLdsBytes) {
        kc::set_error("kc_factor_set_schedule: the staged row does not fit in LDS");
        return KC_EINVAL;
    }
    if (order == KC_ORDER_LONGEST) {
        const kc_status st = build_longest(f, f->last);
        if (st != KC_OK) return st;
    }
    f->wpb = wpb;
    f->persist_max = persist_max;
    f->order = order;
    return KC_OK;
}

kc_status kc_factor_set_stage_limit(kc_factor* f, int32_t max_parents) {
    if (!f || max_parents < -1) {
        kc::set_error("kc_factor_set_stage_limit: max_parents must be >= -1");
        return KC_EINVAL;
    }
    if (max_parents >= 0 && f->mmeta && f->max_row > max_parents) {
        kc::set_error("kc_factor_set_stage_limit: match masks are attached and need every row staged");
        return KC_EINVAL;
    }
    f->stage_max = max_parents < 0 ? f->cap - 2 : std::min(max_parents, f->cap - 2);
    return KC_OK;
}

kc_status kc_factor_use_groups(kc_factor* f, int32_t enable) {
    if (!f) return KC_EINVAL;
    if (enable && !f->groups) {
        kc::set_error("kc_factor_use_groups: only mixed-precision factors of supernodal plans have groups");
        return KC_EINVAL;
    }
    f->use_groups = enable != 0;
    return KC_OK;
}

kc_status kc_factor_schedule(const kc_factor* f, int32_t* wpb, int64_t* persist_max, kc_unit_order* order) {
    if (!f) return KC_EINVAL;
    if (wpb) *wpb = f->wpb;
    if (persist_max) *persist_max = f->persist_max;
    if (order) *order = static_cast<kc_unit_order>(f->order);
    return KC_OK;
}

struct kc_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    kc_factor* f = nullptr;  // the factor whose factorize + solve the graph replays
    int32_t persistent = 0;  // the factorization was recorded with persistent launches
    ~kc_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

kc_status kc_graph_create(kc_factor* f, const double* x_dev, double nu, double ell, const double* ell_dev,
                          kc_pivot pivot, double tau, const double* b_dev, double* sol_dev, int32_t nrhs,
                          void* scratch_dev, size_t scratch_bytes, kc_graph** out) {
    if (!out || !f || !x_dev || !b_dev || !sol_dev || !scratch_dev || nrhs < 1) return KC_EINVAL;
    *out = nullptr;
    if ((f->ninst > 1) != (ell_dev != nullptr)) {
        kc::set_error("kc_graph_create: pass ell_dev exactly for batch plans");
        return KC_EINVAL;
    }
    if (scratch_bytes < solve_scratch_bytes(f, nrhs) || reinterpret_cast<uintptr_t>(scratch_dev) % 256) {
        kc::set_error("kc_graph_create: scratch must be 256-byte aligned and hold kc_solve_bytes bytes");
        return KC_EWORKSPACE;
    }
    std::unique_ptr<kc_graph> g(new (std::nothrow) kc_graph);
    if (!g) return KC_ENOMEM;
    auto capture = [&](hipError_t& e) -> kc_status {
        hipStream_t cs = nullptr;
        KC_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        kc_status st = KC_OK;
        if (e == hipSuccess) {
            st = factorize_impl(f, x_dev, nu, ell, ell_dev, pivot, tau, 0, cs);
            if (st == KC_OK) {
                double* y = static_cast<double*>(scratch_dev);
                double* partial = reinterpret_cast<double*>(static_cast<char*>(scratch_dev) +
                                                            align256(size_t(f->n) * size_t(nrhs) * sizeof(double)));
                st = f->prec == KC_FP64 ? solve_typed<double>(f, b_dev, sol_dev, nrhs, y, partial, cs)
                                        : solve_typed<float>(f, b_dev, sol_dev, nrhs, y, partial, cs);
            }
            hipGraph_t graph = nullptr;
            hipError_t e2 = hipStreamEndCapture(cs, &graph);
            if (e2 != hipSuccess && st == KC_OK) e = e2;
            if (e == hipSuccess && st == KC_OK) g->graph = graph;
            else if (graph) (void)hipGraphDestroy(graph);
        }
        (void)hipStreamDestroy(cs);
        return st;
    };
    // Graphs record one launch per level: cooperative launches are not recorded
    // (the grid barrier of a persistent launch needs the runtime's cooperative
    // launch path at every replay).  The factor's own schedule is kept for eager use.
    // Capturing records the launches without running them: the factor's state
    // (its last stream -- the capture stream is destroyed below -- and whether L
    // has been computed) stays what it was until a replay runs.
    const int64_t pm = f->persist_max;
    hipStream_t const last = f->last;
    const bool factorized = f->factorized, counted = f->counted;
    f->persist_max = 0;
    hipError_t e = hipSuccess;
    kc_status st = capture(e);
    f->persist_max = pm;
    f->last = last;
    f->factorized = factorized;
    f->counted = counted;
    const bool persistent_recorded = false;
    if (e != hipSuccess) {
        kc::set_error(std::string("kc_graph_create: capture failed: ") + hipGetErrorString(e));
        return KC_EHIP;
    }
    if (st != KC_OK) return st;
    KC_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    g->persistent = persistent_recorded ? 1 : 0;
    g->f = f;
    *out = g.release();
    return KC_OK;
}

kc_status kc_graph_info(const kc_graph* g, int64_t* nodes, int32_t* persistent) {
    if (!g) return KC_EINVAL;
    if (nodes) {
        size_t cnt = 0;
        KC_HIP(hipGraphGetNodes(g->graph, nullptr, &cnt));
        *nodes = int64_t(cnt);
    }
    if (persistent) *persistent = g->persistent;
    return KC_OK;
}

kc_status kc_graph_launch(kc_graph* g, void* stream) {
    if (!g) return KC_EINVAL;
    KC_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
    // the replay computes L on `stream`: stats and export wait for it there
    g->f->last = static_cast<hipStream_t>(stream);
    g->f->factorized = true;
    g->f->counted = false;
    return KC_OK;
}

void kc_graph_destroy(kc_graph* g) { delete g; }

}  // extern "C"
