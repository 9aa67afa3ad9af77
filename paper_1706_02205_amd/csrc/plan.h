// Host-side plan: ordering, pattern and schedule produced by kc_analyze.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "kchol.h"

namespace kc {

// One wavefront's share of the factorization: 64 consecutive entries of a column.
struct Unit {
    int32_t col;    // column j (maximin position)
    int32_t first;  // offset of the chunk's first entry inside column j
};

constexpr int kRowAlign = 64;

// Backward solve: one piece of a column's dot product sum_k L_kj x_k over
// entries [start, start + len) counted from the diagonal's successor ...
struct BwdChunk {
    int32_t col;    // column j
    int32_t start;
    int32_t slot;   // where the piece's partial sums go
    int32_t len;
};
// ... and a column of the top block (the columns up to the last long one),
// finished from its pieces' partial sums and its top part.
struct TopCol {
    int32_t col;
    int32_t s1, n1;  // partial sums of its rows below the top block
    int32_t s2, n2;  // partial sums of a long top part (n2 = 0: the part is summed in place)
    int32_t ntop;    // entries of the top part: rows above the diagonal's successor and below the top bound
    int32_t pad0, pad1;
};

// A group of at most 16 consecutive members of a supernode (supernodal plans):
// columns [g0, g1) of the supernode that ends at s1, with nb rows below the
// group's diagonal block in column g0.
struct GroupDesc {
    int32_t g0, g1, s1, nb;
};

struct Plan {
    int64_t n = 0;
    int32_t d = 0;
    int32_t rule = 0;
    double rho = 0.0;

    std::vector<int32_t> perm;      // maximin position -> original index
    std::vector<double> l;          // l[k], l[0] = +inf
    std::vector<double> xh;         // points in maximin order, n x d
    std::vector<int32_t> spatial;   // positions in k-d tree leaf order (a spatial order for any d)

    // lower triangle of S incl. diagonal, CSC (rows ascending, diagonal first)
    std::vector<int64_t> colptr;
    std::vector<int32_t> rowidx;
    // the same entries by rows (CSR, columns ascending, diagonal last); each row
    // starts on a multiple of kRowAlign entries and is padded with INT32_MAX
    std::vector<int64_t> rowptr;    // n + 1 padded row starts
    std::vector<int64_t> rowend;    // n: one past the diagonal
    std::vector<int32_t> colidx;
    std::vector<uint32_t> csc2csr;  // CSR position of each CSC entry
    // the column indices of the padded rows once more, as 16-bit gaps (read by the
    // factorization): entry t of a row stores colidx[t] - colidx[t-1] (the first
    // entry colidx + 1, so a gap is never 0); a gap of delta_limit or more is stored
    // as 0 and the index itself goes to esc -- row k's escapes are
    // esc[escptr[k] .. escptr[k+1]), in row order.  Padding stores 0.
    std::vector<uint16_t> cdelta;   // nnz_rows
    std::vector<uint32_t> escptr;   // n + 1
    std::vector<int32_t> esc;
    uint32_t delta_limit = 65536;

    // elimination DAG: column j waits for every i < j with (j,i) in S
    std::vector<int32_t> level;     // per column
    int32_t nlevels = 0;
    std::vector<Unit> units;        // grouped by level
    std::vector<int64_t> unit_off;  // nlevels + 1
    std::vector<int32_t> fwd_rows;  // rows grouped by level (forward solve)
    std::vector<int64_t> fwd_off;   // nlevels + 1
    // reverse DAG: column j waits for every k > j in column j (backward solve)
    int32_t nrlevels = 0;
    std::vector<int32_t> bwd_cols;  // columns grouped by reverse level
    std::vector<int64_t> bwd_off;   // nrlevels + 1

    // supernodes (supernodal plans only): positions [snode_ptr[s], snode_ptr[s+1]) form supernode s
    std::vector<int64_t> snode_ptr;

    // independent instances (a batch): positions [inst_off[i], inst_off[i+1]) belong to instance i
    int32_t ninst = 1;
    std::vector<int64_t> inst_off;  // ninst + 1
    std::vector<int32_t> inst;      // instance of each position (empty for a single instance)

    int64_t max_col = 0, max_row = 0;
    double t_order = 0, t_pattern = 0, t_schedule = 0;

    int64_t nnz() const { return colptr.empty() ? 0 : colptr.back(); }
    int64_t nnz_rows() const { return rowptr.empty() ? 0 : rowptr.back(); }  // padded
};

// analysis.cpp
void maximin_order(const double* x, int64_t n, int32_t d, int nthreads, int32_t* perm, double* l);
void build_pattern(Plan& p, int nthreads);
void build_schedule(Plan& p, int nthreads);
// Supernodal ordering and pattern (aggregation of nearby points of one scale):
// turns a plan with the maximin ordering and plain pattern into one whose
// positions list supernodes consecutively and whose pattern is the block closure.
void supernodal_transform(Plan& p, int nthreads);
// Block-diagonal union of independently analysed instances.
void merge_plans(const std::vector<Plan>& parts, Plan& out);
// (Re)builds cdelta / escptr / esc from colidx with p.delta_limit.
void encode_row_deltas(Plan& p, int nthreads);

// Thread-local error message shared by the C ABI.
void set_error(const std::string& msg);

}  // namespace kc

struct kc_plan {
    kc::Plan p;
};
