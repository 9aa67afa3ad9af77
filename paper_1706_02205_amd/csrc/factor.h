// Device-side state of one factor (shared by the factorization, solve and PCG sources).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "kchol.h"
#include "plan.h"

struct kc_factor {
    int64_t n = 0, nnz = 0, nnz_rows = 0, nunits = 0;
    int32_t d = 0;
    int32_t cap = 0;          // LDS entries of the staged row (longest row + 2, rounded up)
    int32_t nbuck = 0;        // bucket directory of the staged row (0: cursor merge)
    int32_t max_row = 0;      // longest row of S (parents)
    int32_t stage_max = 0;    // rows with more parents are not staged in LDS (read from device memory)
    int32_t wpb = 4;          // wavefronts per block of the factorization kernel
    int64_t persist_max = 0;  // levels with at most this many units run in persistent launches
    int32_t num_cu = 0;       // compute units of the factor's device
    kc_prec prec = KC_FP64;
    // device regions
    unsigned long long* counters = nullptr;
    double* xh = nullptr;
    int32_t* perm = nullptr;
    int64_t* colptr = nullptr;
    int32_t* rowidx = nullptr;
    uint32_t* csc2csr = nullptr;
    int64_t* rowptr = nullptr;
    int64_t* rowend = nullptr;
    int32_t* colidx = nullptr;
    uint32_t* cdelta = nullptr;  // 16-bit row-index gaps, two per word
    uint32_t* escptr = nullptr;
    int32_t* esc = nullptr;
    void* L = nullptr;        // by rows: double[nnz_rows] or float[nnz_rows]
    void* Lcsc = nullptr;     // by columns: double[nnz] or float[nnz]
    double* diag = nullptr;   // MIXED only
    kc::Unit* units = nullptr;
    int64_t* unit_off_dev = nullptr;  // nlevels + 1, units of each level
    // block units of the factorization for 1, 2 and 4 wavefronts per workgroup:
    // 64 * wpb consecutive entries of one column each, grouped by level, once in
    // each unit order ([order][w], see kc_unit_order)
    kc::Unit* bunits[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
    int32_t order = KC_ORDER_SPATIAL;  // kc_unit_order in use
    // the LONGEST order's own workspace regions; bunits[KC_ORDER_LONGEST] points
    // at SPATIAL's arrays until that order is built (build_longest)
    kc::Unit* bunits_alt[3] = {nullptr, nullptr, nullptr};
    int64_t* boff_dev[3] = {nullptr, nullptr, nullptr};
    std::vector<int64_t> boff[3];
    int32_t* fwd_rows = nullptr;
    int32_t* bwd_short = nullptr;
    kc::TopCol* bwd_top = nullptr;
    kc::BwdChunk* bwd_chunks = nullptr;
    int32_t* inst = nullptr;   // instance of each position (batches only)
    // supernodal groups on the matrix cores (mixed precision, supernodal plans)
    kc::GroupDesc* groups = nullptr;
    int2* gunits = nullptr;
    std::vector<int64_t> goff;
    bool use_groups = false;
    int32_t ninst = 1;
    // host schedule
    std::vector<int64_t> unit_off, fwd_off, short_off, top_off, tchunk_off;
    int64_t nfine = 0;        // pieces of the top columns' rows below the top block (first in bwd_chunks)
    int64_t max_slots = 0;    // partial sums the backward sweep needs at once
    // match masks (kc_factor_match_build), in a caller-owned buffer; null: index merge
    uint64_t* mmeta = nullptr;
    uint64_t* mwords = nullptr;
    uint64_t mwords_n = 0;
    uint64_t match_words = 0;  // mask words the pattern needs, once counted
    bool match_counted = false;
    bool factorized = false;
    bool counted = false;
    hipStream_t last = nullptr;
    // second stream and its event for kc_factorize_solve (created on first use)
    hipStream_t aux = nullptr;
    hipEvent_t aux_ev = nullptr;
};
