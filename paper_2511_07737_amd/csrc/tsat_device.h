// tsat_device.h -- argument blocks shared by the kernels and the host runtime
// of the gradient-guided SAT library.  Internal: not part of the C-ABI.
//
// A solver holds one or more CNF instances (a batch of instances of uneven
// size is stored block-diagonally: instance j owns a contiguous range of
// variables and, inside every width bucket, a contiguous range of clauses).
// Every instance has N candidates; histograms, dL/dR tables and SAT
// bookkeeping are per instance.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tsat.h"
#include "tsat_types.h"

namespace tsat {

// Solver-wide control block in device memory.  The SmoothMin kernel writes
// the schedule scalars of the pending update, the update kernel advances the
// iteration index, so a run of steps (or a captured graph of them) needs no
// host round trip.
struct Ctrl {
    int64_t t;          // next 0-based iteration index
    int64_t updates;    // iterations performed (lifetime)
    double lr;          // learning rate of the pending update
    int32_t stop;       // every instance is frozen: kernels return at entry
    int32_t stop_on_sat;
    int32_t n_frozen;   // instances frozen on a satisfying candidate
    int32_t nonfinite;  // a theta/m/v value became NaN or Inf
    float f_decay;      // 1 - lr * weight_decay
    float f_step;       // lr / (1 - beta1^t)
    float f_isbc2;      // 1 / sqrt(1 - beta2^t)
    float pad0;
    int64_t t_reset;    // iteration at which the AdamW moments last started from zero
    int32_t mixing;     // the pending update is an assignment mixing (no gradient step)
    int32_t pad1;
};

// Per-instance bookkeeping, written by the SmoothMin kernel.
struct InstCtrl {
    int64_t first_sat_step;  // -1 until a candidate satisfies every clause
    int64_t first_conv_step; // -1 until the best candidate passes conv_frac * C
    int64_t best_sat;        // satisfied clauses of the best candidate, last forward
    uint64_t start_time;     // device real-time counter at the first forward
    uint64_t sat_time;       // device real-time counter when first satisfied
    uint64_t conv_time;      // device real-time counter when first converged
    double loss;             // Eq. 3 at the last forward
    int32_t best_cand;
    int32_t sat_cand;        // first satisfying candidate
    int32_t frozen;          // stop_on_sat: no further updates of this instance
    int32_t witness_pending; // the pending update records the satisfying candidate
};

// One forward work unit: a clause range of one instance inside one bucket.
struct FwdUnit {
    int32_t inst;
    int32_t pad;
    int64_t c0, c1;
};

struct FwdArgs {
    const uint32_t* codes;  // [Cb][KW] literal indices of one width bucket
    const FwdUnit* units;   // [gridDim.x]
    int32_t KW;             // clause width of the bucket
    int32_t K1;             // histogram bins (max width + 1)
    const uint32_t* bits32; // literal rows viewed as dwords, row stride W2
    int32_t W2;             // dwords per literal row (2 W)
    int32_t Dn;             // dwords that hold candidates: ceil(N / 32)
    int32_t DT;             // candidate dwords per block tile
    int32_t CPT;            // clauses per thread (<= 255)
    uint32_t* H;            // [n_inst][Np][K1] accumulators
    int64_t H_stride;       // Np * K1
    const Ctrl* ctrl;       // may be null
    const InstCtrl* ictrl;  // may be null
    uint32_t* planes;       // null, or [clauses][plane_P][plane_stride]: R of every clause in binary
    int32_t plane_stride;   // dwords per plane row (2 J, J the update kernel's words per candidate row;
                            // 1 when a clause's two planes share one 8-byte word, N <= 32)
    int32_t plane_P;        // planes per clause (2 or 4)
    int64_t plane_base;     // global index of the bucket's first clause
    int32_t vrows;          // bits32 holds value rows only ([V][W2]); not-x is the complement
    int32_t nunits;         // work units of the launch
    int32_t xcd;            // XCD-aware unit order (grid rounded up to a multiple of 8)
    // KW = 0 (wide-clause kernel): the units of every wide bucket in one
    // launch; a unit's width is in its pad field
    const uint32_t* wide_codes[TSAT_MAX_WIDTH + 1];
    int64_t wide_base[TSAT_MAX_WIDTH + 1];
    // all buckets in one launch (fwd_multi_kernel): codes and plane base of
    // every width in wide_codes / wide_base; the four-plane region (widths
    // 4 and up) starts wide_off dwords after planes
    int64_t wide_off;
};

struct SminArgs {
    uint32_t* H;            // [n_inst][Np][K1] accumulators (read, optionally zeroed)
    uint32_t* H_last;       // [n_inst][N][K1] copy including empty clauses, may be null
    float* table;           // [n_inst][K1][Np] dL/dR, may be null
    float* S_out;           // [n_inst][N] SmoothMin, may be null
    double* S64_out;        // [n_inst][N] SmoothMin in FP64, may be null
    int64_t* sat_out;       // [n_inst][N] satisfied clauses, may be null
    const float* dS;        // [n_inst][N] upstream gradient; null: -dloss, or -1 (Eq. 3)
    const float* dloss;     // [n_inst] upstream gradient of the loss, may be null (1)
    float* loss_out;        // [n_inst] Eq. 3 in FP32, may be null
    Ctrl* ctrl;             // may be null (stateless evaluation)
    InstCtrl* ictrl;        // may be null (stateless evaluation)
    const InstInfo* info;   // [n_inst]
    int32_t n_inst, N, Np, K1;
    int32_t zero_H;
    int32_t update;         // schedule the AdamW update of this step
    int32_t every, restart;
    int32_t mix;            // mix the candidates at learning-rate restarts
    double tau, lr0, decay, lr_min, beta1, beta2, weight_decay, conv_frac;
};

// Levels counted by the mixed-width window gather for a widest clause of K
// literals (one kernel instance per value); its dL/dR table in LDS has
// levels + 1 rows, the rows beyond K zero.
inline int levels_for_width(int K) { return K <= 3 ? 3 : (K <= 4 ? 4 : (K <= 8 ? 8 : (K <= 12 ? 12 : 15))); }

struct VarArgs {
    int32_t V, N, W, Np, K1, mode;
    int32_t lit_rows;         // 1: V rows of logits, each one literal's own row of
                              // bits (independent literal rows); 0: a variable
                              // row writes its value and complement rows
    int32_t pure_k;           // 2..4: every clause has this width and the records
                              // carry no header; 0: generic records
    int32_t group;            // records per scalar-load group in the pure kernel
    int32_t window;           // clause-plane gather by 64-record windows (vector loads, transposed)
    int32_t packed;           // 1: two variables per wave (uniform widths 2 and 3, N <= 32), the
                              // forward's two planes of a clause in one 8-byte word (plane 0 in
                              // the low dword, plane 1 in the high one)
    int32_t xcd;              // XCD-aware order of the variable chunks
    const uint32_t* occ_off;  // [V+1] offsets into occ_data (words, or records if pure)
    const uint32_t* occ_mid;  // [V] first record of negative occurrences
    const uint32_t* occ_data; // records: [k-1,] the other k-1 literal indices
    const uint32_t* var_inst; // [V] instance of each variable, null for one instance
    const uint64_t* lits_cur; // [2V][W] (+16 words of padding)
    uint64_t* lits_next;      // [2V][W]
    const double* mu_cur;     // [V] row means of theta behind lits_cur (raw, unclamped)
    double* mu_next;          // [V] row means written with lits_next
    const float* tbl;         // [n_inst][K1][Np]
    float* theta;
    float* m;
    float* v;
    float* U_out;             // [V][N], may be null
    float* g_out;             // [V][N] or [N][V], may be null
    const float* dA_in;       // [V][N] dL/d(theta_norm) for the Eq. 5 backward op
    uint64_t* vbits_out;      // [V][W] value rows of the binarize op, may be null
    float* assign_out;        // [V][N] 0/1 values of the binarize op, may be null
    int32_t g_transposed;
    float beta1, beta2, one_minus_beta1, one_minus_beta2, eps;
    double inv_n;             // 1 / N (row means and the Eq. 5 backward multiply by it)
    Ctrl* ctrl;
    const InstCtrl* ictrl;    // may be null
    uint8_t* witness;         // [V]
    // clause-plane gather (uniform widths 2 and 3): per variable, positive
    // then negative records holding the clause index (offsets as occ_off /
    // occ_mid), and the forward pass's planes of R for these bits
    const uint32_t* occ_cid;  // null: gather the other literals' rows instead
    const uint32_t* planes;   // [clauses][P][2 J] dwords
    uint32_t narrow_end;      // clauses below this global index hold 2 planes, the rest 4 (after them)
    const uint32_t* cid_off;  // [V+1] record offsets of occ_cid
    const uint32_t* cid_mid;  // [V] first record of negative occurrences
    const uint32_t* vchunk;   // null, or [n_vchunk + 1] first variables of the mixed-width
                              // window gather's work items (at most 8 variables and
                              // 64 records each, or one variable)
    int32_t n_vchunk;
    // generic stores: variables with many occurrence words are split into
    // chunks of records handled by separate waves; their FP64 partial sums
    // are added in chunk order by one wave per variable, which runs the tail
    const uint32_t* heavy;    // [V] 1: handled by the chunk kernels; null: none
    int32_t n_heavy, n_chunks;
    const uint32_t* hv_var;   // [n_heavy]
    const uint32_t* hv_chunk; // [n_heavy + 1] first chunk of each heavy variable
    const uint32_t* ch_var;   // [n_chunks]
    const uint32_t* ch_beg;   // [n_chunks] word range of the chunk's records
    const uint32_t* ch_end;   // [n_chunks]
    double* partial;          // [n_chunks][Np]
};

struct SelectArgs {
    const float* gT;        // [N][V]
    const uint32_t* occ_off;
    const uint64_t* lits;   // [2V][W]
    const int32_t* order;   // candidates by priority
    int32_t V, W, k, kpow2;
    int32_t* lits_out;      // [nblocks][k]
    int32_t* cand_out;      // [nblocks]
};

hipError_t launch_fwd(const FwdArgs& a, int nunits, int tiles, hipStream_t st);
hipError_t launch_fwd_wide(const FwdArgs& a, int kmax, int nunits, int tiles, hipStream_t st);
hipError_t launch_fwd_multi(const FwdArgs& a, int kmax, int nunits, hipStream_t st);
hipError_t launch_planes_hist(const FwdArgs& a, int kmax, int nunits, hipStream_t st);
hipError_t launch_smin(const SminArgs& a, hipStream_t st);
hipError_t launch_adj_scatter(const uint32_t* codes, int64_t Cb, int k, int N, int K1, const uint32_t* bits32,
                              int W2, const float* tbl, float* U, int V, hipStream_t st);
hipError_t launch_fwd_units(FwdUnit* u, int64_t n, int64_t per, int64_t Cb, hipStream_t st);
// device address of the allocation-free entry point's fixed scratch array on
// `device` (which must be current); looked up once per device
hipError_t noalloc_scratch_address(int device, void** out);
hipError_t launch_var(const VarArgs& a, int op, int blocks, hipStream_t st);
int var_occupancy(const VarArgs& a, int op); // resident 256-thread blocks per CU of the step kernel
hipError_t launch_expand(const uint64_t* bits, int64_t V, int W, int N, uint64_t* lits, hipStream_t st);
hipError_t launch_pack(const float* assign, int V, int N, int W, uint64_t* out, int lit_rows, hipStream_t st);
hipError_t launch_init_normal(float* theta, int64_t n, uint64_t seed, hipStream_t st);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t val, hipStream_t st);
hipError_t launch_copy16(void* dst, const void* src, int64_t n16, int blocks, hipStream_t st);
hipError_t launch_stream(int kind, uint32_t* a, uint32_t* b, uint32_t* c, const uint32_t* src, int64_t n4, int blocks,
                         hipStream_t st);
hipError_t launch_strided_rows(const uint64_t* src, int64_t rows, int w, int64_t src_stride, uint64_t* dst,
                               hipStream_t st);
hipError_t launch_rank(const int64_t* sat, int N, int32_t* order, hipStream_t st);
hipError_t launch_select(const SelectArgs& a, int nblocks, hipStream_t st);

enum { VOP_STEP = 0, VOP_GRAD = 1, VOP_ADJ = 2, VOP_BINARIZE = 3, VOP_NORMBWD = 4 };

} // namespace tsat
