// tsat_store.h -- host-side clause and occurrence stores (Sec. III-A: the
// rows of P, one per clause, over the 2V literal columns; Sec. IV-A: P is
// kept sparse).  Plain C++, no HIP: the builder and the DIMACS reader are
// also compiled into a sanitizer-instrumented host test.
#pragma once

#include <stdint.h>

#include <vector>

#include "tsat.h"
#include "tsat_types.h"

namespace tsat_host {

constexpr uint32_t kHeavyWords = 768;
constexpr uint32_t kChunkWords = 512;


// Size limits of the occurrence store.  The record offsets are 32-bit, and
// the header-less records of uniform-width stores are addressed by 32-bit
// byte offsets in the row-gather kernel: a store whose header-less records
// would pass max_pure_bytes is built with generic records instead (the
// kernels reading those use 64-bit addresses).  The margin below 2^32 covers
// the grouped loads that run up to 64 words past a variable's last record.
// Tests shrink the limits.
struct StoreLimits {
    uint64_t max_occ_words = 0xffffffffull;
    uint64_t max_pure_bytes = 0xffffffffull - (1ull << 16);
};

// A batch of instances is stored block-diagonally: instance j's variables
// are var_base[j] .. var_base[j+1]-1 of the union, and inside every width
// bucket its clauses are the contiguous range inst_off[k][j] .. [j+1].
struct Store {
    int32_t V = 0;       // variables of the union
    int32_t K = 0;       // widest clause
    int64_t C = 0;       // clauses including empty ones
    int64_t L = 0;       // literal occurrences
    int64_t n_empty = 0;
    int64_t n_dup = 0;
    int64_t n_taut = 0;
    int64_t width_count[TSAT_MAX_WIDTH + 1] = {0};
    std::vector<std::vector<uint32_t>> buckets; // [k] -> [Cb][k] literal codes 2*var+neg
    int32_t n_inst = 1;
    std::vector<uint32_t> var_base;                // [n_inst+1]
    std::vector<tsat::InstInfo> info;                    // [n_inst]
    std::vector<std::vector<int64_t>> inst_off;    // [k][n_inst+1]
    // Occurrence store.  Generic: per variable, word offsets of records
    // (k-1, other literal codes).  Pure (every non-empty clause of width
    // pure_k in 2..4): record offsets of header-less records of k-1 codes.
    int32_t pure_k = 0;
    std::vector<uint32_t> occ_off, occ_mid, occ_data;
    uint64_t max_sign_deg = 0; // most records of one variable and sign
    // uniform widths 2 and 3: the same records as clause indices within the bucket
    std::vector<uint32_t> occ_cid;
    // generic records: variables with more than kHeavyWords occurrence words,
    // cut at record boundaries into chunks of at most kChunkWords words
    std::vector<uint32_t> heavy, hv_var, hv_chunk, ch_var, ch_beg, ch_end;
};

// Validate n_inst DIMACS streams (instance j: lits[lit_off[j] .. lit_off[j+1]),
// variables 1..num_vars[j]) and build the clause store of their union:
// repeated literals inside a clause are removed, tautologies and empty
// clauses kept, clauses bucketed by width in instance order; with_occ also
// builds the occurrence store.  TSAT_E_ARG / TSAT_E_OOM with the message in
// tsat_last_error's buffer.
int32_t build_store(int32_t n_inst, const int32_t* num_vars, const int64_t* lit_off, const int32_t* lits,
                    Store& st, bool with_occ, const StoreLimits& lim = StoreLimits());

} // namespace tsat_host
