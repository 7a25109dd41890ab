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
// widest clause of a store whose update gathers the forward's planes of R
// (R of a clause in binary: 2 planes up to width 3, 4 up to width 15)
constexpr int32_t kMaxPlaneWidth = 15;
inline int32_t planes_for_width(int32_t K) { return K <= 3 ? 2 : 4; }


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
    // Clause-index records (every store with 1 <= K <= kMaxPlaneWidth and
    // fewer than 2^32 clauses and occurrences): per variable, the global
    // indices of the clauses it occurs in, positive occurrences first; a
    // clause of width k at position c of its bucket has global index
    // plane_base[k] + c.  The record offsets are cid_off / cid_mid, or, in a
    // uniform-width store (whose occurrence records are counted in records
    // too), occ_off / occ_mid (cid_off stays empty).
    std::vector<uint32_t> occ_cid, cid_off, cid_mid;
    std::vector<int64_t> plane_base;   // [TSAT_MAX_WIDTH + 1]; empty without records
    int64_t plane_clauses = 0;         // clauses of widths >= 1 (rows of the plane array)
    uint64_t max_sign_rec = 0;         // most clause-index records of one variable and sign
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

// Work items of a window gather over records with offsets off[0 .. V]:
// the first variables of runs of consecutive variables, each run as long as
// it holds at most max_vars variables and max_records records (a variable
// with more records forms a run alone); the table ends with V.
std::vector<uint32_t> window_chunks(const std::vector<uint32_t>& off, size_t V, size_t max_vars = 8,
                                    uint32_t max_records = 64);

} // namespace tsat_host
