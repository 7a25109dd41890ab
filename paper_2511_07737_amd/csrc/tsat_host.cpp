// tsat_host.cpp -- host runtime and C-ABI of the gfx950 gradient-guided SAT
// library (TurboSAT, arXiv 2511.07737).  Builds the clause and occurrence
// stores, owns device memory, sequences the kernels of each iteration and
// implements every entry point declared in tsat.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "tsat.h"
#include "tsat_device.h"
#include "tsat_host_util.h"
#include "tsat_learned.h"
#include "tsat_store.h"

using namespace tsat;
using namespace tsat_host;

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------

struct Bucket {
    int32_t k;
    int64_t count;
    DBuf codes;
    // forward work units of this bucket, per slot count (256 / DT)
    std::map<int, std::pair<DBuf*, int>> units;
    ~Bucket()
    {
        for (auto& u : units) delete u.second.first;
    }
};

struct tsat_solver {
    int32_t device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    tsat_params params{};
    int32_t cus = 256;

    bool loaded = false;
    Store st;
    std::vector<Bucket*> buckets;
    DBuf occ_off, occ_mid, occ_data, var_inst, info;
    DBuf occ_cid;            // clause-index records (widths up to kMaxPlaneWidth)
    DBuf cid_off, cid_mid;   // their record offsets (stores with generic occurrence records)
    DBuf vchunk;             // work items of the mixed-width window gather: first variables
    int32_t n_vchunk = 0;
    DBuf planes, planes_scr; // R of every clause in binary, for the step / for evaluations
    DBuf heavy, hv_var, hv_chunk, ch_var, ch_beg, ch_end; // chunked heavy variables (generic stores)
    DBuf partial, partial_scr; // FP64 partial sums of the chunks, for the step / for evaluations

    // independent literal rows (one logit row per literal, 2V rows): requested
    // for the next batch, and the layout of the current one (1 or 2 rows per
    // variable); lro: each literal's clause-index record range
    int32_t lit_rows_req = 0;
    int32_t rows_per_var = 1;
    DBuf lro;

    // batch
    int32_t N = 0, W = 0, Np = 0;
    DBuf lits[2];
    DBuf mu[2]; // FP64 row means of theta behind lits[cur] / lits[1-cur]
    int cur = 0;
    int32_t bits_mode = TSAT_MODE_MEAN; // normalization mode the current bits were computed with
    DBuf theta, m, v;
    DBuf H, H_last, table, S64, sat;
    DBuf ctrl, ictrl, ctrl_scr, witness;
    // scratch for stateless evaluations and the device-pointer API
    DBuf lits_scr, mu_scr, H_scr, table_scr, S64_scr, sat_scr, tmp;
    int32_t scr_Np = 0;
    void* noalloc_scratch = nullptr; // this device's fixed scratch array (tsat_fwd_dev_noalloc)
    int32_t noalloc_rc = 0;          // status of its address lookup at creation

    // graph replay of two iterations (one per buffer parity)
    bool use_graph = false;
    hipGraphExec_t graph_exec = nullptr;
    std::vector<char> graph_key;

    // launch shapes (autotuned or set; environment overrides at creation)
    int32_t fwd_target_blocks = 1024; // forward work units per launch to aim for
    int32_t var_per_cu = 0;           // variable-major blocks per CU (0: 4 x occupancy)
    int32_t pure_group = 2;           // records per load group, uniform-width stores
    int32_t clause_planes = 1;        // uniform widths 2, 3: backward gathers the forward's planes of R
    int32_t window_gather = 1;        // clause planes: 64 records per vector load, transposed across the wave
    int32_t xcd_order = 1;            // XCD-aware order of the forward's work units
    int32_t xcd_update = 0;           // XCD-aware order of the update's variable chunks

    // forward work units of all wide buckets (widths > 4) in one launch, per clauses-per-wave
    std::map<int, std::pair<DBuf*, int>> wide_units;
    // forward work units of every bucket in one launch (mixed widths with
    // clause planes), per clauses-per-thread
    std::map<int, std::pair<DBuf*, int>> multi_units;

    // learned proposal: features and aggregation channels, kept proposal
    DBuf feat, fh[2], fzinv, prop;
    bool prop_valid = false;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    double timed_ms[3] = {0, 0, 0};
    int32_t timed_iters = 0;

    void drop_graph()
    {
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        graph_exec = nullptr;
        graph_key.clear();
    }
    ~tsat_solver()
    {
        drop_graph();
        for (auto* b : buckets) delete b;
        for (auto& u : wide_units) delete u.second.first;
        for (auto& u : multi_units) delete u.second.first;
        for (auto e : events) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

static int32_t K1_of(const tsat_solver* s) { return s->st.K + 1; }

// logit rows of the batch: one per variable, or one per literal
static size_t theta_rows(const tsat_solver* s) { return (size_t)s->rows_per_var * s->st.V; }

static int32_t set_dev(tsat_solver* s)
{
    HIPCHK(hipSetDevice(s->device));
    return TSAT_OK;
}

static int32_t validate_params(const tsat_params* p)
{
    if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) return fail(TSAT_E_ARG, "tau must be finite and >= 0");
    if (p->decay_every <= 0 || p->restart_every <= 0) return fail(TSAT_E_ARG, "decay_every and restart_every must be > 0");
    if (!(p->beta1 >= 0 && p->beta1 < 1 && p->beta2 >= 0 && p->beta2 < 1)) return fail(TSAT_E_ARG, "betas must be in [0, 1)");
    if (!(p->eps > 0) || !(p->lr0 >= 0) || !(p->lr_min >= 0)) return fail(TSAT_E_ARG, "eps must be > 0, learning rates >= 0");
    if (p->norm_mode != TSAT_MODE_MEAN && p->norm_mode != TSAT_MODE_NONE) return fail(TSAT_E_ARG, "norm_mode must be 0 or 1");
    if (p->mix != 0 && p->mix != 1) return fail(TSAT_E_ARG, "mix must be 0 or 1");
    return TSAT_OK;
}

// Forward launch geometry of one width bucket for N candidates: DT candidate
// dwords per block (LDS bins <= 64 KiB), S = 256/DT clause slots, up to 255
// clauses per thread (8-plane counters), units sized for ~target blocks.
struct FwdGeom {
    int DT, S, CPT, tiles, Dn;
};

static FwdGeom fwd_geometry(int32_t N, int32_t K1, int64_t Cb, int32_t KW, int32_t target_blocks)
{
    FwdGeom g;
    g.Dn = (N + 31) / 32;
    if (KW > 4) {
        // wide clauses: blocks of four waves, each wave a run of CPT clauses
        // for 64 candidates; about four waves per targeted block in all
        g.DT = 2;
        g.S = 4;
        g.tiles = (N + 63) / 64;
        const int64_t waves = 4 * (int64_t)std::max(1, target_blocks);
        const int64_t cpt = (Cb * g.tiles + waves - 1) / waves;
        g.CPT = (int)std::max<int64_t>(8, std::min<int64_t>(1024, cpt));
        return g;
    }
    const int bins = KW + 1;
    g.DT = std::min(g.Dn, 64);
    while (g.DT > 1 && (size_t)g.DT * 32 * bins * 4 > 64 * 1024) g.DT >>= 1;
    g.S = 256 / g.DT;
    g.tiles = (g.Dn + g.DT - 1) / g.DT;
    target_blocks = std::max(1, target_blocks);
    const int64_t target_x = std::max<int64_t>(1, (target_blocks + g.tiles - 1) / g.tiles);
    int64_t cpt = (Cb + (int64_t)g.S * target_x - 1) / ((int64_t)g.S * target_x);
    g.CPT = (int)std::max<int64_t>(16, std::min<int64_t>(255, cpt));
    return g;
}

// Work units of a bucket for a slot count: per instance, clause ranges of at
// most S * CPT clauses (a unit never spans two instances).
static int32_t bucket_units(tsat_solver* s, Bucket* b, const FwdGeom& g, const FwdUnit** out, int* count)
{
    const int key = g.S * 1000 + g.CPT;
    auto it = b->units.find(key);
    if (it == b->units.end()) {
        std::vector<FwdUnit> u;
        const int64_t per = (int64_t)g.S * g.CPT;
        const auto& off = s->st.inst_off[b->k];
        for (int32_t j = 0; j < s->st.n_inst; ++j)
            for (int64_t c = off[j]; c < off[j + 1]; c += per) u.push_back(FwdUnit{j, 0, c, std::min(c + per, off[j + 1])});
        DBuf* d = new (std::nothrow) DBuf();
        if (!d) return fail(TSAT_E_OOM, "host allocation failed");
        int32_t rc = d->alloc(std::max<size_t>(1, u.size()) * sizeof(FwdUnit), "forward units");
        if (rc) { delete d; return rc; }
        if (!u.empty()) {
            hipError_t e = hipMemcpy(d->p, u.data(), u.size() * sizeof(FwdUnit), hipMemcpyHostToDevice);
            if (e != hipSuccess) { delete d; return fail(TSAT_E_HIP, "unit upload: %s", hipGetErrorString(e)); }
        }
        it = b->units.emplace(key, std::make_pair(d, (int)u.size())).first;
    }
    *out = it->second.first->as<FwdUnit>();
    *count = it->second.second;
    return TSAT_OK;
}

// Make every bucket's unit table for N candidates resident (before a graph
// capture, which must not allocate or copy).
static int32_t wide_geometry(const tsat_solver* s, int32_t N, FwdGeom* g, int* kmax);
static int32_t wide_units(tsat_solver* s, const FwdGeom& g, const FwdUnit** out, int* count);
static bool multi_path(const tsat_solver* s, int32_t N);
static FwdGeom multi_geometry(const tsat_solver* s, int32_t N, int* kmax);
static int32_t multi_units(tsat_solver* s, const FwdGeom& g, const FwdUnit** out, int* count);

static int32_t prepare_units(tsat_solver* s, int32_t N)
{
    if (multi_path(s, N)) {
        int kmax;
        const FwdGeom g = multi_geometry(s, N, &kmax);
        const FwdUnit* u;
        int n;
        RET(multi_units(s, g, &u, &n));
    }
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0 || b->k > 4) continue;
        const FwdGeom g = fwd_geometry(N, K1_of(s), b->count, b->k, s->fwd_target_blocks);
        const FwdUnit* u;
        int n;
        RET(bucket_units(s, b, g, &u, &n));
    }
    FwdGeom g;
    int kmax;
    if (wide_geometry(s, N, &g, &kmax)) {
        const FwdUnit* u;
        int n;
        RET(wide_units(s, g, &u, &n));
    }
    return TSAT_OK;
}

// enqueue the forward histograms of every width bucket on literal rows `lits`
// Words per candidate row the update kernels use for W words (a power of two).
static int32_t row_words(int32_t W) { return W <= 2 ? W : (W <= 4 ? 4 : (W <= 8 ? 8 : 16)); }

static bool uniform_plane_store(const tsat_solver* s) { return s->st.pure_k == 2 || s->st.pure_k == 3; }

// LDS of the mixed-width window gather: four windows of P J 64 words and one
// dL/dR table of (levels + 1) J 64 floats per block (one instance) or per
// wave (batch)
static size_t levels_lds_bytes(const tsat_solver* s, int32_t J)
{
    const size_t P = (size_t)planes_for_width(s->st.K);
    const size_t rows = (size_t)levels_for_width(s->st.K) + 1;
    return 4 * P * J * 64 * 8 + (s->st.n_inst > 1 ? 4 : 1) * rows * J * 64 * 4;
}

// The clause-plane update applies: clause-index records exist (widths up to
// kMaxPlaneWidth), at most 256 candidates, and, beyond uniform widths 2 and
// 3 (which also have a record-by-record plane gather), the window gather
// with its 16-bit counts and LDS budget.
static bool plane_path(const tsat_solver* s, int32_t N)
{
    if (!s->clause_planes || !s->occ_cid.p || (N + 63) / 64 > 4) return false;
    if (uniform_plane_store(s)) return true;
    return s->window_gather && s->st.max_sign_rec < 65536 && levels_lds_bytes(s, row_words((N + 63) / 64)) <= 65536;
}

// Uniform widths 2 and 3 with the window gather at N <= 32: the update takes
// two variables per wave and reads a clause's two planes as one 8-byte word,
// so the forward writes them packed (plane stride of one dword).  The one
// predicate sets the forward's layout and picks the update kernel.
static bool packed_planes(const tsat_solver* s, int32_t N)
{
    return N <= 32 && s->rows_per_var == 1 && uniform_plane_store(s) && s->window_gather &&
           s->st.max_sign_rec < 65536 && plane_path(s, N);
}

// Planes of R for N candidates: [clauses][P][2 J] dwords, zeroed when (re)allocated.
// Clauses of widths 1 .. 3 come first in the global clause order and hold
// two planes each (R <= 3); the wider ones follow with four.
static int64_t narrow_end(const tsat_solver* s)
{
    return s->st.K >= 4 ? s->st.plane_base[4] : s->st.plane_clauses;
}

static int32_t ensure_planes(tsat_solver* s, DBuf& buf, int32_t N, hipStream_t st)
{
    const size_t G3 = (size_t)narrow_end(s);
    const size_t words = G3 * 2 + ((size_t)s->st.plane_clauses - G3) * 4; // plane rows
    const size_t bytes = std::max<size_t>(16, words * 8 * (size_t)row_words((N + 63) / 64));
    if (buf.p && buf.bytes >= bytes) return TSAT_OK;
    RET(buf.alloc(bytes, "clause planes"));
    HIPCHK(launch_fill_u32(buf.as<uint32_t>(), (int64_t)(bytes / 4), 0u, st));
    return TSAT_OK;
}

// Work units of every wide bucket (width > 4) for one launch of the
// wide-clause kernel: per bucket and instance, ranges of 4 CPT clauses
// (a unit never spans two buckets or instances); the width goes in pad.
static int32_t wide_geometry(const tsat_solver* s, int32_t N, FwdGeom* g, int* kmax)
{
    int64_t Cw = 0;
    *kmax = 0;
    for (auto* b : s->buckets)
        if (b->k > 4 && b->count > 0) {
            Cw += b->count;
            *kmax = std::max(*kmax, b->k);
        }
    *g = fwd_geometry(N, K1_of(s), Cw, 5, s->fwd_target_blocks);
    return Cw > 0;
}

static int32_t wide_units(tsat_solver* s, const FwdGeom& g, const FwdUnit** out, int* count)
{
    auto it = s->wide_units.find(g.CPT);
    if (it == s->wide_units.end()) {
        std::vector<FwdUnit> u;
        const int64_t per = (int64_t)g.S * g.CPT;
        for (auto* b : s->buckets) {
            if (b->k <= 4 || b->count == 0) continue;
            const auto& off = s->st.inst_off[b->k];
            for (int32_t j = 0; j < s->st.n_inst; ++j)
                for (int64_t c = off[j]; c < off[j + 1]; c += per)
                    u.push_back(FwdUnit{j, b->k, c, std::min(c + per, off[j + 1])});
        }
        DBuf* d = new (std::nothrow) DBuf();
        if (!d) return fail(TSAT_E_OOM, "host allocation failed");
        int32_t rc = d->alloc(std::max<size_t>(1, u.size()) * sizeof(FwdUnit), "forward units");
        if (rc) { delete d; return rc; }
        if (!u.empty()) {
            hipError_t e = hipMemcpy(d->p, u.data(), u.size() * sizeof(FwdUnit), hipMemcpyHostToDevice);
            if (e != hipSuccess) { delete d; return fail(TSAT_E_HIP, "unit upload: %s", hipGetErrorString(e)); }
        }
        it = s->wide_units.emplace(g.CPT, std::make_pair(d, (int)u.size())).first;
    }
    *out = it->second.first->as<FwdUnit>();
    *count = it->second.second;
    return TSAT_OK;
}

// Every bucket of a store with two or more non-empty widths in one forward
// launch: clause planes on (so at most 256 candidates, one tile per block).
static bool multi_path(const tsat_solver* s, int32_t N)
{
    if (!plane_path(s, N)) return false;
    int nb = 0;
    for (auto* b : s->buckets)
        if (b->k > 0 && b->count > 0) ++nb;
    return nb >= 2;
}

static FwdGeom multi_geometry(const tsat_solver* s, int32_t N, int* kmax)
{
    int64_t C = 0;
    *kmax = 0;
    for (auto* b : s->buckets)
        if (b->k > 0 && b->count > 0) {
            C += b->count;
            *kmax = std::max(*kmax, b->k);
        }
    return fwd_geometry(N, K1_of(s), C, 4, s->fwd_target_blocks);
}

// per bucket (width in pad) and instance, ranges of S CPT clauses
static int32_t multi_units(tsat_solver* s, const FwdGeom& g, const FwdUnit** out, int* count)
{
    auto it = s->multi_units.find(g.CPT);
    if (it == s->multi_units.end()) {
        std::vector<FwdUnit> u;
        const int64_t per = (int64_t)g.S * g.CPT;
        for (auto* b : s->buckets) {
            if (b->k == 0 || b->count == 0) continue;
            const auto& off = s->st.inst_off[b->k];
            for (int32_t j = 0; j < s->st.n_inst; ++j)
                for (int64_t c = off[j]; c < off[j + 1]; c += per)
                    u.push_back(FwdUnit{j, b->k, c, std::min(c + per, off[j + 1])});
        }
        DBuf* d = new (std::nothrow) DBuf();
        if (!d) return fail(TSAT_E_OOM, "host allocation failed");
        int32_t rc = d->alloc(std::max<size_t>(1, u.size()) * sizeof(FwdUnit), "forward units");
        if (rc) { delete d; return rc; }
        if (!u.empty()) {
            hipError_t e = hipMemcpy(d->p, u.data(), u.size() * sizeof(FwdUnit), hipMemcpyHostToDevice);
            if (e != hipSuccess) { delete d; return fail(TSAT_E_HIP, "unit upload: %s", hipGetErrorString(e)); }
        }
        it = s->multi_units.emplace(g.CPT, std::make_pair(d, (int)u.size())).first;
    }
    *out = it->second.first->as<FwdUnit>();
    *count = it->second.second;
    return TSAT_OK;
}

static int32_t enqueue_fwd(tsat_solver* s, const uint64_t* lits, int32_t N, uint32_t* H, const Ctrl* ctrl,
                           const InstCtrl* ictrl, hipStream_t st, uint32_t* planes = nullptr)
{
    const int32_t W = (N + 63) / 64;
    const bool with_planes = planes && plane_path(s, N);
    FwdArgs base{};
    base.K1 = K1_of(s);
    base.bits32 = reinterpret_cast<const uint32_t*>(lits);
    base.W2 = 2 * W;
    base.H = H;
    base.H_stride = (int64_t)64 * W * base.K1;
    base.ctrl = ctrl;
    base.ictrl = ictrl;
    // narrow clauses (widths 1 .. 3): two planes each from the start of the
    // plane buffer; wider ones: four planes each after them
    const int64_t G3 = with_planes ? narrow_end(s) : 0;
    uint32_t* wide_planes = nullptr;
    if (with_planes) {
        base.planes = planes;
        base.plane_stride = packed_planes(s, N) ? 1 : 2 * row_words(W);
        wide_planes = planes + (size_t)G3 * 2 * base.plane_stride;
    }
    if (with_planes && multi_path(s, N)) {
        // every bucket in one launch, then the wide clauses' histogram pass
        int kmax = 0;
        const FwdGeom g = multi_geometry(s, N, &kmax);
        FwdArgs a = base;
        int nunits = 0;
        RET(multi_units(s, g, &a.units, &nunits));
        a.KW = 0;
        a.Dn = g.Dn;
        a.DT = g.DT;
        a.CPT = g.CPT;
        a.plane_P = 2;
        a.wide_off = (int64_t)G3 * 2 * base.plane_stride;
        for (auto* b : s->buckets) {
            if (b->k == 0 || b->count == 0) continue;
            a.wide_codes[b->k] = b->codes.as<uint32_t>();
            a.wide_base[b->k] = s->st.plane_base[b->k] - (b->k <= 3 ? 0 : G3);
        }
        a.nunits = nunits;
        a.xcd = s->xcd_order;
        if (nunits > 0) HIPCHK(launch_fwd_multi(a, kmax, nunits, st));
        FwdGeom gw;
        int kw = 0;
        if (wide_geometry(s, N, &gw, &kw)) {
            FwdArgs w = a;
            int nw = 0;
            RET(wide_units(s, gw, &w.units, &nw));
            w.CPT = gw.CPT;
            w.planes = wide_planes;
            w.plane_P = 4;
            w.nunits = nw;
            if (nw > 0) HIPCHK(launch_planes_hist(w, kw, nw, st));
        }
        return TSAT_OK;
    }
    // widths 1 .. 4: one launch per bucket
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0 || b->k > 4) continue;
        const FwdGeom g = fwd_geometry(N, K1_of(s), b->count, b->k, s->fwd_target_blocks);
        FwdArgs a = base;
        int nunits = 0;
        RET(bucket_units(s, b, g, &a.units, &nunits));
        if (nunits == 0) continue;
        a.codes = b->codes.as<uint32_t>();
        a.KW = b->k;
        a.Dn = g.Dn;
        a.DT = g.DT;
        a.CPT = g.CPT;
        if (with_planes) {
            const bool narrow = b->k <= 3;
            a.planes = narrow ? planes : wide_planes;
            a.plane_P = narrow ? 2 : 4;
            a.plane_base = s->st.plane_base[b->k] - (narrow ? 0 : G3);
        }
        a.nunits = nunits;
        a.xcd = s->xcd_order;
        HIPCHK(launch_fwd(a, nunits, g.tiles, st));
    }
    // wider clauses: every bucket in one launch
    FwdGeom g;
    int kmax = 0;
    if (wide_geometry(s, N, &g, &kmax)) {
        FwdArgs a = base;
        int nunits = 0;
        RET(wide_units(s, g, &a.units, &nunits));
        a.KW = 0;
        a.Dn = g.Dn;
        a.DT = g.DT;
        a.CPT = g.CPT;
        if (with_planes) {
            a.planes = wide_planes;
            a.plane_P = 4;
        }
        for (auto* b : s->buckets) {
            if (b->k <= 4 || b->count == 0) continue;
            a.wide_codes[b->k] = b->codes.as<uint32_t>();
            if (with_planes) a.wide_base[b->k] = s->st.plane_base[b->k] - G3;
        }
        a.nunits = nunits;
        a.xcd = s->xcd_order;
        if (nunits > 0) HIPCHK(launch_fwd_wide(a, kmax, nunits, g.tiles, st));
    }
    return TSAT_OK;
}

static SminArgs smin_args(tsat_solver* s, const tsat_params& p, int32_t N, int32_t Np)
{
    SminArgs a{};
    a.info = s->info.as<InstInfo>();
    a.n_inst = s->st.n_inst;
    a.N = N;
    a.Np = Np;
    a.K1 = K1_of(s);
    a.zero_H = 1;
    a.every = p.decay_every;
    a.restart = p.restart_every;
    a.mix = p.mix;
    a.tau = p.tau;
    a.lr0 = p.lr0;
    a.decay = p.lr_decay;
    a.lr_min = p.lr_min;
    a.beta1 = p.beta1;
    a.beta2 = p.beta2;
    a.weight_decay = p.weight_decay;
    a.conv_frac = p.converge_frac;
    return a;
}

// Persistent variable-major kernels: by default as many blocks as the CUs
// hold at the kernel's occupancy, times 4 (measured faster than exactly one
// resident round: waves that finish early pick up the remaining blocks).
static int var_blocks(const tsat_solver* s, int32_t V, int occ = 0)
{
    const int per_cu = s->var_per_cu > 0 ? s->var_per_cu : (occ > 0 ? 4 * occ : 32);
    const int64_t want = ((int64_t)V + 3) / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)s->cus * per_cu));
}

static VarArgs var_args(tsat_solver* s, const tsat_params& p, int32_t N, int32_t W, int32_t Np)
{
    VarArgs a{};
    a.V = s->st.V;
    a.N = N;
    a.W = W;
    a.Np = Np;
    a.inv_n = 1.0 / (double)N;
    a.K1 = K1_of(s);
    a.mode = p.norm_mode;
    a.pure_k = s->st.pure_k;
    a.group = s->pure_group;
    // the window gather keeps its counts in 16-bit halves
    a.window = s->window_gather && s->st.max_sign_rec < 65536;
    a.packed = packed_planes(s, N);
    a.xcd = s->xcd_update;
    a.occ_off = s->occ_off.as<uint32_t>();
    a.occ_mid = s->occ_mid.as<uint32_t>();
    a.occ_data = s->occ_data.as<uint32_t>();
    a.var_inst = s->st.n_inst > 1 ? s->var_inst.as<uint32_t>() : nullptr;
    a.beta1 = (float)p.beta1;
    a.beta2 = (float)p.beta2;
    a.one_minus_beta1 = (float)(1.0 - p.beta1);
    a.one_minus_beta2 = (float)(1.0 - p.beta2);
    a.eps = (float)p.eps;
    // clause-plane gather: evaluations write their planes to planes_scr, the
    // step overrides this with its own buffer
    a.occ_cid = plane_path(s, N) ? s->occ_cid.as<uint32_t>() : nullptr;
    a.narrow_end = s->loaded && s->occ_cid.p ? (uint32_t)narrow_end(s) : 0u;
    a.cid_off = s->cid_off.p ? s->cid_off.as<uint32_t>() : a.occ_off;
    a.cid_mid = s->cid_mid.p ? s->cid_mid.as<uint32_t>() : a.occ_mid;
    a.vchunk = s->vchunk.p ? s->vchunk.as<uint32_t>() : nullptr;
    a.n_vchunk = s->n_vchunk;
    a.planes = s->planes_scr.as<uint32_t>();
    if (s->heavy.p) {
        a.heavy = s->heavy.as<uint32_t>();
        a.n_heavy = (int32_t)s->st.hv_var.size();
        a.n_chunks = (int32_t)s->st.ch_var.size();
        a.hv_var = s->hv_var.as<uint32_t>();
        a.hv_chunk = s->hv_chunk.as<uint32_t>();
        a.ch_var = s->ch_var.as<uint32_t>();
        a.ch_beg = s->ch_beg.as<uint32_t>();
        a.ch_end = s->ch_end.as<uint32_t>();
        a.partial = s->partial_scr.as<double>(); // evaluations; the step uses its own buffer
    }
    return a;
}

// The batch's own update launches: with independent literal rows the rows
// are the 2V literals, each gathering its own clause-index records (all
// counted as positive occurrences: lro[l] .. lro[l + 1]).
static void batch_rows(const tsat_solver* s, VarArgs& a)
{
    if (s->rows_per_var != 2) return;
    a.V = 2 * s->st.V;
    a.lit_rows = 1;
    a.occ_off = a.cid_off = s->lro.as<uint32_t>();
    a.vchunk = nullptr; // built over the variables' records, not the literals'
    a.occ_mid = a.cid_mid = s->lro.as<uint32_t>() + 1;
    a.var_inst = nullptr;
    a.window = 1;
    a.packed = 0;
}

// FP64 partial rows of the heavy-variable chunks for N candidates
static int32_t ensure_partial(tsat_solver* s, DBuf& buf, int32_t N)
{
    if (!s->heavy.p) return TSAT_OK;
    return buf.reserve(s->st.ch_var.size() * (size_t)(64 * ((N + 63) / 64)) * sizeof(double), "chunk partial sums");
}

// the variable-major kernels address literal rows with 32-bit byte offsets
static int32_t check_row_offsets(const tsat_solver* s, int32_t W)
{
    const uint64_t bytes = (uint64_t)2 * s->st.V * W * 8;
    if (bytes > 0xffffffffull)
        return fail(TSAT_E_ARG, "2V * ceil(N/64) * 8 = %llu bytes exceeds the 32-bit row offsets", (unsigned long long)bytes);
    return TSAT_OK;
}

static int32_t ensure_scratch(tsat_solver* s, int32_t N)
{
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    const int32_t K1 = K1_of(s);
    const size_t ni = (size_t)s->st.n_inst;
    RET(s->lits_scr.reserve(((size_t)2 * s->st.V * W + 16) * 8, "scratch literal rows"));
    RET(s->mu_scr.reserve((size_t)s->st.V * 8, "scratch row means"));
    if (Np > s->scr_Np) {
        RET(s->H_scr.alloc(ni * Np * K1 * 4, "scratch histogram"));
        HIPCHK(launch_fill_u32(s->H_scr.as<uint32_t>(), (int64_t)(ni * Np * K1), 0u, s->stream));
        // the device-pointer calls run on the caller's stream: finish the fill first
        HIPCHK(hipStreamSynchronize(s->stream));
        RET(s->table_scr.alloc(ni * Np * K1 * 4, "scratch table"));
        RET(s->S64_scr.alloc(ni * Np * 8, "scratch S"));
        RET(s->sat_scr.alloc(ni * Np * 8, "scratch sat counts"));
        s->scr_Np = Np;
    }
    return TSAT_OK;
}

static int32_t reset_ctrl(tsat_solver* s, int64_t t)
{
    Ctrl c{};
    c.t = t;
    HIPCHK(hipMemcpyAsync(s->ctrl.p, &c, sizeof c, hipMemcpyHostToDevice, s->stream));
    std::vector<InstCtrl> ic((size_t)s->st.n_inst);
    for (auto& x : ic) {
        x = InstCtrl{};
        x.first_sat_step = -1;
        x.first_conv_step = -1;
        x.sat_cand = -1;
    }
    HIPCHK(hipMemcpyAsync(s->ictrl.p, ic.data(), ic.size() * sizeof(InstCtrl), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

static int32_t binarize_current(tsat_solver* s, int32_t mode)
{
    tsat_params p = s->params;
    p.norm_mode = mode;
    VarArgs a = var_args(s, p, s->N, s->W, s->Np);
    a.lits_next = s->lits[s->cur].as<uint64_t>();
    a.mu_next = s->mu[s->cur].as<double>();
    a.theta = s->theta.as<float>();
    a.ctrl = s->ctrl.as<Ctrl>();
    batch_rows(s, a);
    HIPCHK(launch_var(a, VOP_BINARIZE, var_blocks(s, a.V), s->stream));
    s->bits_mode = mode;
    return TSAT_OK;
}

// the bits of the batch follow the normalization mode of the call using them
static int32_t ensure_mode(tsat_solver* s, int32_t mode)
{
    if (s->bits_mode == mode) return TSAT_OK;
    return binarize_current(s, mode);
}

static int32_t read_ictrl(tsat_solver* s, std::vector<InstCtrl>& out)
{
    out.resize((size_t)s->st.n_inst);
    HIPCHK(hipMemcpyAsync(out.data(), s->ictrl.p, out.size() * sizeof(InstCtrl), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* tsat_last_error(void) { return g_err.c_str(); }

int32_t tsat_version(void) { return 10100; }

int32_t tsat_default_params(tsat_params* p)
{
    if (!p) return fail(TSAT_E_ARG, "params pointer is NULL");
    p->tau = 1.0;
    p->lr0 = 0.1;
    p->lr_decay = 0.1;
    p->lr_min = 1e-15;
    p->beta1 = 0.9;
    p->beta2 = 0.999;
    p->eps = 1e-8;
    p->weight_decay = 1e-2;
    p->converge_frac = 0.99;
    p->decay_every = 30;
    p->restart_every = 360;
    p->norm_mode = TSAT_MODE_MEAN;
    p->k_partial = 0;
    p->mix = 0;
    p->reserved = 0;
    return TSAT_OK;
}

int32_t tsat_create(const tsat_config* cfg, tsat_solver** out)
{
    g_err.clear();
    if (!out) return fail(TSAT_E_ARG, "out is NULL");
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || count == 0) {
        (void)hipGetLastError();
        return fail(TSAT_E_HIP, "no HIP device available");
    }
    const int dev = cfg ? cfg->device : 0;
    if (dev < 0 || dev >= count) return fail(TSAT_E_ARG, "device %d out of range (%d devices)", dev, count);
    tsat_solver* s = new (std::nothrow) tsat_solver();
    if (!s) return fail(TSAT_E_OOM, "host allocation failed");
    s->device = dev;
    if (cfg) {
        s->params = cfg->params;
        int32_t rc = validate_params(&s->params);
        if (rc) { delete s; return rc; }
    } else {
        tsat_default_params(&s->params);
    }
    if (hipSetDevice(dev) != hipSuccess) { delete s; return fail(TSAT_E_HIP, "hipSetDevice(%d) failed", dev); }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess && prop.multiProcessorCount > 0) s->cus = prop.multiProcessorCount;
    // device address of the fixed scratch array, once per device (with it current)
    {
        const hipError_t e = noalloc_scratch_address(dev, &s->noalloc_scratch);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            s->noalloc_scratch = nullptr;
            s->noalloc_rc = (int32_t)e;
        }
    }
    s->fwd_target_blocks = std::max(1, env_int("TSAT_FWD_TARGET_BLOCKS", s->fwd_target_blocks));
    s->var_per_cu = std::max(0, env_int("TSAT_VAR_BLOCKS_PER_CU", s->var_per_cu));
    s->pure_group = env_int("TSAT_PURE_GROUP", s->pure_group);
    s->clause_planes = env_int("TSAT_CLAUSE_PLANES", s->clause_planes) != 0;
    s->window_gather = env_int("TSAT_WINDOW_GATHER", s->window_gather) != 0;
    s->xcd_order = env_int("TSAT_XCD_ORDER", s->xcd_order) != 0;
    s->xcd_update = env_int("TSAT_XCD_UPDATE", s->xcd_update) != 0;
    if (cfg && cfg->stream) {
        s->stream = (hipStream_t)cfg->stream;
    } else {
        if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess) {
            delete s;
            return fail(TSAT_E_HIP, "stream creation failed");
        }
        s->own_stream = true;
    }
    int32_t rc = s->ctrl.alloc(sizeof(Ctrl), "control block");
    if (!rc) rc = s->ctrl_scr.alloc(sizeof(Ctrl), "scratch control block");
    if (rc) { delete s; return rc; }
    const Ctrl zero{};
    if (hipMemcpy(s->ctrl_scr.p, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(s->ctrl.p, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) {
        delete s;
        return fail(TSAT_E_HIP, "control block initialization failed");
    }
    *out = s;
    return TSAT_OK;
}

void tsat_destroy(tsat_solver* s)
{
    if (!s) return;
    (void)hipSetDevice(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    delete s;
}

static int32_t load_store(tsat_solver* s, Store&& st)
{
    HIPCHK(hipStreamSynchronize(s->stream));
    s->drop_graph();
    for (auto* b : s->buckets) delete b;
    s->buckets.clear();
    for (auto& u : s->wide_units) delete u.second.first;
    s->wide_units.clear();
    for (auto& u : s->multi_units) delete u.second.first;
    s->multi_units.clear();
    s->loaded = false;
    s->lit_rows_req = 0;
    s->rows_per_var = 1;
    s->lro.release();
    s->N = s->W = s->Np = 0;
    s->scr_Np = 0;
    s->prop_valid = false;
    s->st = std::move(st);
    for (int k = 0; k <= s->st.K; ++k) {
        const auto& codes = s->st.buckets[k];
        const int64_t cnt = s->st.width_count[k];
        if (cnt == 0) continue;
        Bucket* b = new (std::nothrow) Bucket();
        if (!b) return fail(TSAT_E_OOM, "host allocation failed");
        b->k = k;
        b->count = cnt;
        s->buckets.push_back(b);
        if (k == 0) continue;
        RET(b->codes.alloc(codes.size() * 4, "clause store"));
        HIPCHK(hipMemcpy(b->codes.p, codes.data(), codes.size() * 4, hipMemcpyHostToDevice));
    }
    const size_t V = (size_t)s->st.V;
    RET(s->occ_off.alloc((V + 1) * 4, "occurrence offsets"));
    RET(s->occ_mid.alloc(V * 4, "occurrence offsets"));
    HIPCHK(hipMemcpy(s->occ_off.p, s->st.occ_off.data(), (V + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->occ_mid.p, s->st.occ_mid.data(), V * 4, hipMemcpyHostToDevice));
    // 64 zero words of padding: grouped record loads near the end stay in bounds
    const size_t occ_words = s->st.occ_data.size();
    RET(s->occ_data.alloc((occ_words + 64) * 4, "occurrence records"));
    HIPCHK(launch_fill_u32(s->occ_data.as<uint32_t>() + occ_words, 64, 0u, s->stream));
    if (occ_words) HIPCHK(hipMemcpy(s->occ_data.p, s->st.occ_data.data(), occ_words * 4, hipMemcpyHostToDevice));
    s->occ_cid.release();
    if (!s->st.occ_cid.empty()) {
        const size_t nr = s->st.occ_cid.size();
        RET(s->occ_cid.alloc((nr + 64) * 4, "clause-index records"));
        HIPCHK(launch_fill_u32(s->occ_cid.as<uint32_t>() + nr, 64, 0u, s->stream));
        HIPCHK(hipMemcpy(s->occ_cid.p, s->st.occ_cid.data(), nr * 4, hipMemcpyHostToDevice));
    }
    s->cid_off.release();
    s->cid_mid.release();
    if (!s->st.cid_off.empty()) {
        RET(s->cid_off.alloc((V + 1) * 4, "clause-index record offsets"));
        RET(s->cid_mid.alloc(std::max<size_t>(1, V) * 4, "clause-index record offsets"));
        HIPCHK(hipMemcpy(s->cid_off.p, s->st.cid_off.data(), (V + 1) * 4, hipMemcpyHostToDevice));
        if (V) HIPCHK(hipMemcpy(s->cid_mid.p, s->st.cid_mid.data(), V * 4, hipMemcpyHostToDevice));
    }
    // work items of the mixed-width window gather: runs of consecutive
    // variables whose records fill one 64-record window (at most 8
    // variables; a variable with more records alone)
    s->vchunk.release();
    s->n_vchunk = 0;
    if (!s->st.cid_off.empty() && V > 0) {
        const std::vector<uint32_t> ch = window_chunks(s->st.cid_off, V);
        RET(s->vchunk.alloc(ch.size() * 4, "variable chunks"));
        HIPCHK(hipMemcpy(s->vchunk.p, ch.data(), ch.size() * 4, hipMemcpyHostToDevice));
        s->n_vchunk = (int32_t)ch.size() - 1;
    }
    s->planes.release();
    s->planes_scr.release();
    s->partial.release();
    s->partial_scr.release();
    {
        const Store& t = s->st;
        DBuf* bufs[] = {&s->heavy, &s->hv_var, &s->hv_chunk, &s->ch_var, &s->ch_beg, &s->ch_end};
        const std::vector<uint32_t>* src[] = {&t.heavy, &t.hv_var, &t.hv_chunk, &t.ch_var, &t.ch_beg, &t.ch_end};
        for (int i = 0; i < 6; ++i) {
            bufs[i]->release();
            if (src[i]->empty()) continue;
            RET(bufs[i]->alloc(src[i]->size() * 4, "heavy-variable chunks"));
            HIPCHK(hipMemcpy(bufs[i]->p, src[i]->data(), src[i]->size() * 4, hipMemcpyHostToDevice));
        }
    }
    const size_t ni = (size_t)s->st.n_inst;
    RET(s->info.alloc(ni * sizeof(InstInfo), "instance sizes"));
    HIPCHK(hipMemcpy(s->info.p, s->st.info.data(), ni * sizeof(InstInfo), hipMemcpyHostToDevice));
    RET(s->ictrl.alloc(ni * sizeof(InstCtrl), "instance control"));
    if (ni > 1) {
        std::vector<uint32_t> vi(V);
        for (size_t j = 0; j < ni; ++j)
            for (uint32_t v = s->st.var_base[j]; v < s->st.var_base[j + 1]; ++v) vi[v] = (uint32_t)j;
        RET(s->var_inst.alloc(V * 4, "variable instances"));
        HIPCHK(hipMemcpy(s->var_inst.p, vi.data(), V * 4, hipMemcpyHostToDevice));
    }
    RET(s->witness.alloc(V, "witness"));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->loaded = true;
    return TSAT_OK;
}

int32_t tsat_load_cnf(tsat_solver* s, int32_t num_vars, int64_t num_lits, const int32_t* lits)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (num_lits < 0) return fail(TSAT_E_ARG, "invalid literal stream (n=%lld)", (long long)num_lits);
    RET(set_dev(s));
    Store st;
    const int64_t off[2] = {0, num_lits};
    RET(build_store(1, &num_vars, off, lits, st, true));
    return load_store(s, std::move(st));
}

int32_t tsat_load_cnf_batch(tsat_solver* s, int32_t n_inst, const int32_t* num_vars, const int64_t* lit_offsets,
                            const int32_t* lits)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (n_inst < 1 || !num_vars || !lit_offsets) return fail(TSAT_E_ARG, "invalid instance list");
    if (lit_offsets[0] != 0) return fail(TSAT_E_ARG, "lit_offsets[0] must be 0");
    for (int32_t j = 0; j < n_inst; ++j)
        if (lit_offsets[j + 1] < lit_offsets[j]) return fail(TSAT_E_ARG, "lit_offsets must be non-decreasing");
    RET(set_dev(s));
    Store st;
    RET(build_store(n_inst, num_vars, lit_offsets, lits, st, true));
    return load_store(s, std::move(st));
}

int32_t tsat_load_dimacs(tsat_solver* s, const char* path)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    int32_t V = 0;
    int64_t n = 0;
    RET(tsat_dimacs_read(path, &V, &n, nullptr, 0));
    std::vector<int32_t> buf;
    try {
        buf.resize((size_t)std::max<int64_t>(n, 1));
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed");
    }
    RET(tsat_dimacs_read(path, &V, &n, buf.data(), n));
    return tsat_load_cnf(s, V, n, buf.data());
}

static int32_t alloc_batch(tsat_solver* s, int32_t N)
{
    const int32_t W = (N + 63) / 64, Np = 64 * W, K1 = K1_of(s);
    if (s->lit_rows_req) {
        // independent literal rows run only on the window gather of the
        // forward's clause planes
        if (!plane_path(s, N))
            return fail(TSAT_E_ARG, "independent literal rows need the clause-plane window gather: N <= 256, "
                                    "clauses at most %d wide, clause planes and the window gather on", kMaxPlaneWidth);
    }
    s->rows_per_var = s->lit_rows_req ? 2 : 1;
    const size_t VN = theta_rows(s) * N;
    const size_t ni = (size_t)s->st.n_inst;
    if ((size_t)K1 * Np * 4 > 64 * 1024)
        return fail(TSAT_E_ARG, "(max_width+1) * 64*ceil(N/64) * 4 bytes = %zu exceeds the 64 KiB table limit",
                    (size_t)K1 * Np * 4);
    RET(check_row_offsets(s, W));
    s->drop_graph();
    // 16 words of padding: the variable-major kernels read whole J-word rows
    const size_t lit_words = (size_t)2 * s->st.V * W + 16;
    for (int b = 0; b < 2; ++b) {
        RET(s->lits[b].alloc(lit_words * 8, "literal rows"));
        HIPCHK(launch_fill_u32(s->lits[b].as<uint32_t>(), (int64_t)lit_words * 2, 0u, s->stream));
        RET(s->mu[b].alloc(theta_rows(s) * 8, "row means"));
    }
    RET(s->theta.alloc(VN * 4, "theta"));
    RET(s->m.alloc(VN * 4, "m"));
    RET(s->v.alloc(VN * 4, "v"));
    RET(s->H.alloc(ni * Np * K1 * 4, "histogram"));
    RET(s->H_last.alloc(ni * Np * K1 * 4, "histogram"));
    RET(s->table.alloc(ni * Np * K1 * 4, "table"));
    RET(s->S64.alloc(ni * Np * 8, "S"));
    RET(s->sat.alloc(ni * Np * 8, "sat counts"));
    HIPCHK(launch_fill_u32(s->H.as<uint32_t>(), (int64_t)(ni * Np * K1), 0u, s->stream));
    HIPCHK(launch_fill_u32(s->H_last.as<uint32_t>(), (int64_t)(ni * Np * K1), 0u, s->stream));
    HIPCHK(launch_fill_u32(s->m.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
    HIPCHK(launch_fill_u32(s->v.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
    if (plane_path(s, N)) RET(ensure_planes(s, s->planes, N, s->stream));
    RET(ensure_partial(s, s->partial, N));
    s->N = N;
    s->W = W;
    s->Np = Np;
    s->cur = 0;
    return TSAT_OK;
}

int32_t tsat_init_batch(tsat_solver* s, int32_t N, uint64_t seed, const float* init_logits)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || N > TSAT_MAX_STEP_N) return fail(TSAT_E_ARG, "N must be in [1, %d] (got %d)", TSAT_MAX_STEP_N, N);
    RET(set_dev(s));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->N = 0;
    RET(alloc_batch(s, N));
    const size_t VN = theta_rows(s) * N;
    if (init_logits) HIPCHK(hipMemcpyAsync(s->theta.p, init_logits, VN * 4, hipMemcpyHostToDevice, s->stream));
    else HIPCHK(launch_init_normal(s->theta.as<float>(), (int64_t)VN, seed, s->stream));
    RET(binarize_current(s, s->params.norm_mode));
    RET(reset_ctrl(s, 0));
    return TSAT_OK;
}

// Features of every variable of the loaded CNF into X[V][16] on stream st:
// round 0 (counts, base features, h0), then three aggregation rounds.
static int32_t enqueue_features(tsat_solver* s, float* X, hipStream_t st)
{
    const size_t V = (size_t)s->st.V;
    RET(s->fh[0].reserve(V * sizeof(float4), "feature channels"));
    RET(s->fh[1].reserve(V * sizeof(float4), "feature channels"));
    RET(s->fzinv.reserve(V * sizeof(float), "feature normalizers"));
    FeatArgs a{};
    a.V = s->st.V;
    a.pure_k = s->st.pure_k;
    a.occ_off = s->occ_off.as<uint32_t>();
    a.occ_mid = s->occ_mid.as<uint32_t>();
    a.occ_data = s->occ_data.as<uint32_t>();
    a.zinv = s->fzinv.as<float>();
    a.X = X;
    for (int r = 0; r <= 3; ++r) {
        a.round = r;
        a.h_prev = s->fh[(r + 1) & 1].as<float4>();
        a.h_next = s->fh[r & 1].as<float4>();
        HIPCHK(launch_features(a, st));
    }
    return TSAT_OK;
}

static int32_t need_loaded(tsat_solver* s)
{
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    return set_dev(s);
}

int32_t tsat_get_features(tsat_solver* s, float* X)
{
    g_err.clear();
    RET(need_loaded(s));
    if (!X) return fail(TSAT_E_ARG, "X is NULL");
    const size_t n = (size_t)s->st.V * kFeat;
    RET(s->feat.reserve(n * sizeof(float), "features"));
    RET(enqueue_features(s, s->feat.as<float>(), s->stream));
    HIPCHK(hipMemcpyAsync(X, s->feat.p, n * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

int32_t tsat_features_dev(tsat_solver* s, float* X, void* stream)
{
    g_err.clear();
    RET(need_loaded(s));
    if (!X) return fail(TSAT_E_ARG, "X is NULL");
    const hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    // scratch channels are shared with the solver's stream: order both ways
    HIPCHK(hipStreamSynchronize(s->stream));
    RET(enqueue_features(s, X, st));
    return TSAT_OK;
}

int32_t tsat_propose(tsat_solver* s, tsat_mlp* m, float* p)
{
    g_err.clear();
    RET(need_loaded(s));
    MlpDev d;
    int32_t dev = -1;
    RET(mlp_view(m, &d, &dev));
    if (dev != s->device) return fail(TSAT_E_ARG, "the network lives on device %d, the solver on %d", dev, s->device);
    const size_t V = (size_t)s->st.V;
    RET(s->feat.reserve(V * kFeat * sizeof(float), "features"));
    RET(s->prop.reserve(V * sizeof(float), "proposal"));
    // the network's buffers are written by the null stream in its set-up calls
    HIPCHK(hipDeviceSynchronize());
    RET(enqueue_features(s, s->feat.as<float>(), s->stream));
    HIPCHK(launch_mlp_forward(d, s->feat.as<float>(), (int64_t)V, nullptr, s->prop.as<float>(), s->stream));
    if (p) HIPCHK(hipMemcpyAsync(p, s->prop.p, V * sizeof(float), hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->prop_valid = true;
    return TSAT_OK;
}

int32_t tsat_init_from_proposal(tsat_solver* s, int32_t N, uint64_t seed, const float* p_true)
{
    g_err.clear();
    RET(need_loaded(s));
    if (N < 1 || N > TSAT_MAX_STEP_N) return fail(TSAT_E_ARG, "N must be in [1, %d] (got %d)", TSAT_MAX_STEP_N, N);
    if (!p_true && !s->prop_valid) return fail(TSAT_E_STATE, "no proposal: pass p_true or call tsat_propose first");
    if (s->lit_rows_req) return fail(TSAT_E_STATE, "the proposal start draws complete assignments (literal rows are on)");
    HIPCHK(hipStreamSynchronize(s->stream));
    const size_t V = (size_t)s->st.V;
    if (p_true) {
        RET(s->prop.reserve(V * sizeof(float), "proposal"));
        HIPCHK(hipMemcpyAsync(s->prop.p, p_true, V * sizeof(float), hipMemcpyHostToDevice, s->stream));
        s->prop_valid = true;
    }
    s->N = 0;
    RET(alloc_batch(s, N));
    PropArgs a{};
    a.V = s->st.V;
    a.N = N;
    a.seed = seed;
    a.mode = s->params.norm_mode;
    a.p = s->prop.as<float>();
    a.theta = s->theta.as<float>();
    HIPCHK(launch_init_proposal(a, s->stream));
    RET(binarize_current(s, s->params.norm_mode));
    RET(reset_ctrl(s, 0));
    return TSAT_OK;
}

static int32_t need_batch(tsat_solver* s)
{
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (s->N <= 0) return fail(TSAT_E_STATE, "no batch: call tsat_init_batch first");
    return set_dev(s);
}

static int32_t need_single(tsat_solver* s)
{
    if (s->st.n_inst != 1) return fail(TSAT_E_STATE, "this call needs a single-instance solver (%d instances loaded)", s->st.n_inst);
    return TSAT_OK;
}

// Enqueue one iteration (forward of all buckets -> SmoothMin -> fused update)
// on literal buffer parity `cur`.
static int32_t enqueue_iteration(tsat_solver* s, const SminArgs& sa, VarArgs va, int vblocks, int cur, bool timing, int it)
{
    Ctrl* ctrl = s->ctrl.as<Ctrl>();
    InstCtrl* ictrl = s->ictrl.as<InstCtrl>();
    RET(enqueue_fwd(s, s->lits[cur].as<uint64_t>(), s->N, s->H.as<uint32_t>(), ctrl, ictrl, s->stream,
                    plane_path(s, s->N) ? s->planes.as<uint32_t>() : nullptr));
    if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 1], s->stream));
    HIPCHK(launch_smin(sa, s->stream));
    if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 2], s->stream));
    va.lits_cur = s->lits[cur].as<uint64_t>();
    va.lits_next = s->lits[1 - cur].as<uint64_t>();
    va.mu_cur = s->mu[cur].as<double>();
    va.mu_next = s->mu[1 - cur].as<double>();
    HIPCHK(launch_var(va, VOP_STEP, vblocks, s->stream));
    if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 3], s->stream));
    return TSAT_OK;
}

int32_t tsat_step(tsat_solver* s, int32_t max_steps, const tsat_params* params, int32_t stop_on_sat, tsat_report* report)
{
    g_err.clear();
    RET(need_batch(s));
    if (max_steps < 0) return fail(TSAT_E_ARG, "max_steps must be >= 0");
    tsat_params p = params ? *params : s->params;
    RET(validate_params(&p));
    RET(ensure_mode(s, p.norm_mode));
    Ctrl* ctrl = s->ctrl.as<Ctrl>();
    // stop flag and its arming for this call
    Ctrl host{};
    HIPCHK(hipMemcpyAsync(&host, ctrl, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    const int64_t updates0 = host.updates;
    host.stop = 0;
    host.stop_on_sat = stop_on_sat == 2 ? 2 : (stop_on_sat ? 1 : 0);
    HIPCHK(hipMemcpyAsync(ctrl, &host, sizeof host, hipMemcpyHostToDevice, s->stream));

    SminArgs sa = smin_args(s, p, s->N, s->Np);
    sa.H = s->H.as<uint32_t>();
    sa.H_last = s->H_last.as<uint32_t>();
    sa.table = s->table.as<float>();
    sa.S64_out = s->S64.as<double>();
    sa.sat_out = s->sat.as<int64_t>();
    sa.ctrl = ctrl;
    sa.ictrl = s->ictrl.as<InstCtrl>();
    sa.update = 1;
    VarArgs va = var_args(s, p, s->N, s->W, s->Np);
    va.planes = s->planes.as<uint32_t>();
    if (va.heavy) va.partial = s->partial.as<double>();
    va.tbl = s->table.as<float>();
    va.theta = s->theta.as<float>();
    va.m = s->m.as<float>();
    va.v = s->v.as<float>();
    va.ctrl = ctrl;
    va.ictrl = s->ictrl.as<InstCtrl>();
    va.witness = s->witness.as<uint8_t>();
    batch_rows(s, va);
    const int vblocks = var_blocks(s, va.V, var_occupancy(va, VOP_STEP));
    RET(prepare_units(s, s->N));

    const bool graph = s->use_graph && !s->timing;
    const bool timing = s->timing && max_steps > 0;
    if (timing) {
        const size_t need = (size_t)3 * max_steps + 1;
        while (s->events.size() < need) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            s->events.push_back(e);
        }
        HIPCHK(hipEventRecord(s->events[0], s->stream));
    }
    int32_t executed = 0;
    if (graph && max_steps >= 2) {
        // capture two iterations (both buffer parities) once per argument set
        std::vector<char> key(sizeof sa + sizeof va + sizeof(int) * 2);
        memcpy(key.data(), &sa, sizeof sa);
        memcpy(key.data() + sizeof sa, &va, sizeof va);
        memcpy(key.data() + sizeof sa + sizeof va, &vblocks, sizeof(int));
        memcpy(key.data() + sizeof sa + sizeof va + sizeof(int), &s->cur, sizeof(int));
        if (!s->graph_exec || key != s->graph_key) {
            s->drop_graph();
            hipGraph_t g;
            HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
            int32_t rc = enqueue_iteration(s, sa, va, vblocks, s->cur, false, 0);
            if (!rc) rc = enqueue_iteration(s, sa, va, vblocks, 1 - s->cur, false, 0);
            hipError_t e = hipStreamEndCapture(s->stream, &g);
            if (rc) return rc;
            if (e != hipSuccess) return fail(TSAT_E_HIP, "graph capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&s->graph_exec, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) {
                s->graph_exec = nullptr;
                return fail(TSAT_E_HIP, "graph instantiation: %s", hipGetErrorString(e));
            }
            s->graph_key = key;
        }
        while (executed + 2 <= max_steps) {
            HIPCHK(hipGraphLaunch(s->graph_exec, s->stream));
            executed += 2;
            if (stop_on_sat && (executed % 16) == 0 && executed < max_steps) {
                HIPCHK(hipMemcpyAsync(&host, ctrl, sizeof host, hipMemcpyDeviceToHost, s->stream));
                HIPCHK(hipStreamSynchronize(s->stream));
                if (host.stop) break;
            }
        }
    }
    for (int32_t it = executed; it < max_steps; ++it) {
        ++executed;
        RET(enqueue_iteration(s, sa, va, vblocks, s->cur, timing, it));
        s->cur = 1 - s->cur;
        if (stop_on_sat && (it % 16) == 15 && it + 1 < max_steps) {
            HIPCHK(hipMemcpyAsync(&host, ctrl, sizeof host, hipMemcpyDeviceToHost, s->stream));
            HIPCHK(hipStreamSynchronize(s->stream));
            if (host.stop) break;
        }
    }
    HIPCHK(hipMemcpyAsync(&host, ctrl, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (timing) {
        double acc[3] = {0, 0, 0};
        int32_t n = 0;
        for (int32_t it = 0; it < executed; ++it) {
            float ms[3];
            bool ok = true;
            for (int k = 0; k < 3; ++k)
                if (hipEventElapsedTime(&ms[k], s->events[3 * it + k], s->events[3 * it + k + 1]) != hipSuccess) ok = false;
            if (!ok) { (void)hipGetLastError(); break; }
            for (int k = 0; k < 3; ++k) acc[k] += ms[k];
            ++n;
        }
        for (int k = 0; k < 3; ++k) s->timed_ms[k] = n ? acc[k] / n : 0.0;
        s->timed_iters = n;
    }
    if (report) {
        std::vector<InstCtrl> ic;
        RET(read_ictrl(s, ic));
        tsat_report r{};
        r.steps_done = host.updates - updates0;
        r.next_step = host.t;
        r.nonfinite = host.nonfinite;
        r.first_sat_step = -1;
        r.first_converged_step = -1;
        r.sat_candidate = ic[0].sat_cand;
        r.best_candidate = ic[0].best_cand;
        for (const auto& x : ic) {
            r.loss += x.loss;
            r.best_sat_count += x.best_sat;
            if (x.first_sat_step >= 0 && (r.first_sat_step < 0 || x.first_sat_step < r.first_sat_step))
                r.first_sat_step = x.first_sat_step;
            if (x.first_conv_step >= 0 && (r.first_converged_step < 0 || x.first_conv_step < r.first_converged_step))
                r.first_converged_step = x.first_conv_step;
        }
        *report = r;
    }
    if (host.nonfinite) return fail(TSAT_E_NUMERIC, "a logit or optimizer moment became non-finite");
    return TSAT_OK;
}

int32_t tsat_set_graph(tsat_solver* s, int32_t enable)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    s->use_graph = enable != 0;
    if (!s->use_graph) s->drop_graph();
    return TSAT_OK;
}

int32_t tsat_num_instances(const tsat_solver* s) { return (s && s->loaded) ? s->st.n_inst : 0; }

int32_t tsat_get_instance_status(tsat_solver* s, int32_t first, int32_t count, tsat_instance_status* out)
{
    g_err.clear();
    RET(need_batch(s));
    if (first < 0 || count < 0 || first + count > s->st.n_inst || (count > 0 && !out))
        return fail(TSAT_E_ARG, "instance range [%d, %d) outside [0, %d)", first, first + count, s->st.n_inst);
    std::vector<InstCtrl> ic;
    RET(read_ictrl(s, ic));
    for (int32_t j = 0; j < count; ++j) {
        const InstCtrl& x = ic[(size_t)(first + j)];
        tsat_instance_status o{};
        o.first_sat_step = x.first_sat_step;
        o.first_converged_step = x.first_conv_step;
        o.best_sat_count = x.best_sat;
        o.num_clauses = s->st.info[(size_t)(first + j)].C;
        o.loss = x.loss;
        o.start_ticks = x.start_time;
        o.sat_ticks = x.sat_time;
        o.conv_ticks = x.conv_time;
        o.best_candidate = x.best_cand;
        o.sat_candidate = x.sat_cand;
        o.frozen = x.frozen;
        o.num_vars = (int32_t)(s->st.var_base[(size_t)(first + j) + 1] - s->st.var_base[(size_t)(first + j)]);
        out[j] = o;
    }
    return TSAT_OK;
}

int32_t tsat_device_clock_hz(tsat_solver* s, double* hz)
{
    g_err.clear();
    if (!s || !hz) return fail(TSAT_E_ARG, "NULL argument");
    int khz = 0;
    HIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device));
    *hz = 1e3 * (double)khz;
    return TSAT_OK;
}

// stateless forward + SmoothMin of literal rows `lits` (N candidates)
static int32_t eval_rows(tsat_solver* s, const tsat_params& p, const uint64_t* lits, int32_t N, const float* dS,
                         uint32_t* H_out, float* S32, double* S64, int64_t* sat, float* table, hipStream_t st,
                         float* loss_out = nullptr, const float* dloss = nullptr)
{
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    uint32_t* planes = nullptr;
    if (plane_path(s, N)) {
        RET(ensure_planes(s, s->planes_scr, N, st));
        planes = s->planes_scr.as<uint32_t>();
    }
    RET(ensure_partial(s, s->partial_scr, N));
    RET(enqueue_fwd(s, lits, N, s->H_scr.as<uint32_t>(), nullptr, nullptr, st, planes));
    SminArgs a = smin_args(s, p, N, Np);
    a.H = s->H_scr.as<uint32_t>();
    a.H_last = H_out;
    a.table = table;
    a.S_out = S32;
    a.S64_out = S64;
    a.sat_out = sat;
    a.dS = dS;
    a.dloss = dloss;
    a.loss_out = loss_out;
    a.update = 0;
    HIPCHK(launch_smin(a, st));
    return TSAT_OK;
}

static int32_t copy_sat(tsat_solver* s, int32_t N, int64_t* sat_counts, uint8_t* is_sat)
{
    const size_t ni = (size_t)s->st.n_inst;
    std::vector<int64_t> sat;
    try {
        sat.resize(ni * (size_t)N);
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed");
    }
    HIPCHK(hipMemcpyAsync(sat.data(), s->sat_scr.p, sat.size() * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (size_t j = 0; j < ni; ++j)
        for (int32_t i = 0; i < N; ++i) {
            const size_t e = j * (size_t)N + (size_t)i;
            if (sat_counts) sat_counts[e] = sat[e];
            if (is_sat) is_sat[e] = sat[e] == s->st.info[j].C ? 1 : 0;
        }
    return TSAT_OK;
}

int32_t tsat_check(tsat_solver* s, int64_t* sat_counts, uint8_t* is_sat)
{
    g_err.clear();
    RET(need_batch(s));
    RET(ensure_scratch(s, s->N));
    RET(eval_rows(s, s->params, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, nullptr, nullptr, nullptr,
                  s->sat_scr.as<int64_t>(), nullptr, s->stream));
    return copy_sat(s, s->N, sat_counts, is_sat);
}

int32_t tsat_check_bits(tsat_solver* s, const uint64_t* packed, int32_t N, int64_t* sat_counts, uint8_t* is_sat)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || !packed) return fail(TSAT_E_ARG, "N must be >= 1 and packed non-NULL");
    RET(set_dev(s));
    const int32_t W = (N + 63) / 64;
    if ((size_t)s->st.n_inst * K1_of(s) * 64 * W * 4 > (size_t)1 << 34) return fail(TSAT_E_ARG, "N too large");
    RET(ensure_scratch(s, N));
    const size_t vb = (size_t)s->st.V * W * 8;
    RET(s->tmp.reserve(vb, "packed input"));
    HIPCHK(hipMemcpyAsync(s->tmp.p, packed, vb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(launch_expand(s->tmp.as<uint64_t>(), s->st.V, W, N, s->lits_scr.as<uint64_t>(), s->stream));
    RET(eval_rows(s, s->params, s->lits_scr.as<uint64_t>(), N, nullptr, nullptr, nullptr, nullptr, s->sat_scr.as<int64_t>(),
                  nullptr, s->stream));
    return copy_sat(s, N, sat_counts, is_sat);
}

int32_t tsat_get_bits(tsat_solver* s, uint64_t* packed)
{
    g_err.clear();
    RET(need_batch(s));
    if (!packed) return fail(TSAT_E_ARG, "packed is NULL");
    if (s->rows_per_var == 2) { // every literal row
        HIPCHK(hipMemcpyAsync(packed, s->lits[s->cur].p, (size_t)2 * s->st.V * s->W * 8, hipMemcpyDeviceToHost,
                              s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
        return TSAT_OK;
    }
    // even literal rows hold the variable values: pack them on the device,
    // then one contiguous copy
    const size_t n = (size_t)s->st.V * s->W;
    RET(s->tmp.reserve(n * 8, "bit staging"));
    HIPCHK(launch_strided_rows(s->lits[s->cur].as<uint64_t>(), s->st.V, s->W, (int64_t)2 * s->W, s->tmp.as<uint64_t>(),
                               s->stream));
    HIPCHK(hipMemcpyAsync(packed, s->tmp.p, n * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

static int32_t column_values(tsat_solver* s, int32_t cand, uint32_t v0, uint32_t v1, uint8_t* vals)
{
    if (s->rows_per_var == 2) return fail(TSAT_E_STATE, "independent literal rows hold no complete assignment");
    const size_t n = v1 - v0;
    std::vector<uint64_t> col(n);
    if (n) {
        RET(s->tmp.reserve(n * 8, "bit staging"));
        HIPCHK(launch_strided_rows(s->lits[s->cur].as<uint64_t>() + (size_t)2 * v0 * s->W + (cand >> 6), (int64_t)n, 1,
                                   (int64_t)2 * s->W, s->tmp.as<uint64_t>(), s->stream));
        HIPCHK(hipMemcpyAsync(col.data(), s->tmp.p, n * 8, hipMemcpyDeviceToHost, s->stream));
        HIPCHK(hipStreamSynchronize(s->stream));
    }
    for (size_t v = 0; v < n; ++v) vals[v] = (uint8_t)((col[v] >> (cand & 63)) & 1u);
    return TSAT_OK;
}

int32_t tsat_get_assignment(tsat_solver* s, int32_t cand, uint8_t* vals)
{
    g_err.clear();
    RET(need_batch(s));
    if (cand < 0 || cand >= s->N || !vals) return fail(TSAT_E_ARG, "candidate %d outside [0, %d) or NULL output", cand, s->N);
    return column_values(s, cand, 0, (uint32_t)s->st.V, vals);
}

int32_t tsat_get_witness_instance(tsat_solver* s, int32_t inst, uint8_t* vals, int32_t* cand)
{
    g_err.clear();
    RET(need_batch(s));
    if (inst < 0 || inst >= s->st.n_inst) return fail(TSAT_E_ARG, "instance %d outside [0, %d)", inst, s->st.n_inst);
    std::vector<InstCtrl> ic;
    RET(read_ictrl(s, ic));
    const InstCtrl& x = ic[(size_t)inst];
    if (x.sat_cand < 0) return fail(TSAT_E_STATE, "no satisfying assignment found yet for instance %d", inst);
    if (cand) *cand = x.sat_cand;
    if (!vals) return TSAT_OK;
    const uint32_t v0 = s->st.var_base[(size_t)inst], v1 = s->st.var_base[(size_t)inst + 1];
    // a frozen instance still holds the satisfying candidate; otherwise the
    // update of the step that found it recorded it
    if (x.frozen || s->rows_per_var == 2) return column_values(s, x.sat_cand, v0, v1, vals);
    HIPCHK(hipMemcpy(vals, s->witness.as<uint8_t>() + v0, v1 - v0, hipMemcpyDeviceToHost));
    return TSAT_OK;
}

int32_t tsat_get_witness(tsat_solver* s, uint8_t* vals, int32_t* cand)
{
    g_err.clear();
    RET(need_batch(s));
    RET(need_single(s));
    return tsat_get_witness_instance(s, 0, vals, cand);
}

int32_t tsat_num_candidates(const tsat_solver* s) { return s ? s->N : 0; }

int32_t tsat_max_width(const tsat_solver* s) { return (s && s->loaded) ? s->st.K : 0; }

int32_t tsat_num_vars(const tsat_solver* s) { return (s && s->loaded) ? s->st.V : 0; }

int32_t tsat_set_logits(tsat_solver* s, const float* theta)
{
    g_err.clear();
    RET(need_batch(s));
    if (!theta) return fail(TSAT_E_ARG, "theta is NULL");
    HIPCHK(hipMemcpyAsync(s->theta.p, theta, theta_rows(s) * s->N * 4, hipMemcpyHostToDevice, s->stream));
    RET(binarize_current(s, s->params.norm_mode));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

int32_t tsat_get_logits(tsat_solver* s, float* theta) { return tsat_get_state(s, theta, nullptr, nullptr, nullptr); }

int32_t tsat_set_state(tsat_solver* s, const float* theta, const float* m, const float* v, int64_t t)
{
    g_err.clear();
    RET(need_batch(s));
    if (!theta || t < 0) return fail(TSAT_E_ARG, "theta is NULL or t < 0");
    const size_t VN = theta_rows(s) * s->N;
    HIPCHK(hipMemcpyAsync(s->theta.p, theta, VN * 4, hipMemcpyHostToDevice, s->stream));
    if (m) HIPCHK(hipMemcpyAsync(s->m.p, m, VN * 4, hipMemcpyHostToDevice, s->stream));
    else HIPCHK(launch_fill_u32(s->m.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
    if (v) HIPCHK(hipMemcpyAsync(s->v.p, v, VN * 4, hipMemcpyHostToDevice, s->stream));
    else HIPCHK(launch_fill_u32(s->v.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
    RET(binarize_current(s, s->params.norm_mode));
    RET(reset_ctrl(s, t));
    return TSAT_OK;
}

int32_t tsat_get_state(tsat_solver* s, float* theta, float* m, float* v, int64_t* t)
{
    g_err.clear();
    RET(need_batch(s));
    const size_t VN = theta_rows(s) * s->N;
    if (theta) HIPCHK(hipMemcpyAsync(theta, s->theta.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    if (m) HIPCHK(hipMemcpyAsync(m, s->m.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    if (v) HIPCHK(hipMemcpyAsync(v, s->v.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    Ctrl host{};
    HIPCHK(hipMemcpyAsync(&host, s->ctrl.p, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (t) *t = host.t;
    return TSAT_OK;
}

int32_t tsat_get_adam_origin(tsat_solver* s, int64_t* origin)
{
    g_err.clear();
    RET(need_batch(s));
    if (!origin) return fail(TSAT_E_ARG, "origin is NULL");
    RET(set_dev(s));
    Ctrl c;
    HIPCHK(hipMemcpyAsync(&c, s->ctrl.p, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    *origin = c.t_reset;
    return TSAT_OK;
}

int32_t tsat_set_adam_origin(tsat_solver* s, int64_t origin)
{
    g_err.clear();
    RET(need_batch(s));
    RET(set_dev(s));
    Ctrl c;
    HIPCHK(hipMemcpyAsync(&c, s->ctrl.p, sizeof c, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (origin < 0 || origin > c.t) return fail(TSAT_E_ARG, "origin must be in [0, %lld]", (long long)c.t);
    c.t_reset = origin;
    HIPCHK(hipMemcpyAsync(s->ctrl.p, &c, sizeof c, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->drop_graph();
    return TSAT_OK;
}

int32_t tsat_eval(tsat_solver* s, const tsat_params* params, uint32_t* hist, double* S, double* loss)
{
    g_err.clear();
    RET(need_batch(s));
    tsat_params p = params ? *params : s->params;
    RET(validate_params(&p));
    RET(ensure_mode(s, p.norm_mode));
    RET(ensure_scratch(s, s->N));
    const int32_t K1 = K1_of(s);
    const size_t ni = (size_t)s->st.n_inst;
    RET(s->tmp.reserve(ni * s->N * K1 * 4, "histogram copy"));
    RET(eval_rows(s, p, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, s->tmp.as<uint32_t>(), nullptr,
                  s->S64_scr.as<double>(), nullptr, nullptr, s->stream));
    std::vector<double> S64(ni * s->N);
    HIPCHK(hipMemcpyAsync(S64.data(), s->S64_scr.p, S64.size() * 8, hipMemcpyDeviceToHost, s->stream));
    if (hist) HIPCHK(hipMemcpyAsync(hist, s->tmp.p, ni * s->N * K1 * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (S) memcpy(S, S64.data(), S64.size() * 8);
    if (loss) {
        // Eq. 3, summed over the candidates of every instance in index order
        double l = 0.0;
        for (double x : S64) l -= x;
        *loss = l;
    }
    return TSAT_OK;
}

int32_t tsat_get_grad(tsat_solver* s, const tsat_params* params, float* U, float* g)
{
    g_err.clear();
    RET(need_batch(s));
    tsat_params p = params ? *params : s->params;
    RET(validate_params(&p));
    RET(ensure_mode(s, p.norm_mode));
    RET(ensure_scratch(s, s->N));
    const size_t VN = theta_rows(s) * s->N;
    RET(s->tmp.reserve(VN * 8, "gradient copies"));
    RET(eval_rows(s, p, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, nullptr, nullptr, nullptr, nullptr,
                  s->table_scr.as<float>(), s->stream));
    VarArgs va = var_args(s, p, s->N, s->W, s->Np);
    va.tbl = s->table_scr.as<float>();
    va.theta = s->theta.as<float>();
    va.lits_cur = s->lits[s->cur].as<uint64_t>();
    va.mu_cur = s->mu[s->cur].as<double>();
    va.U_out = s->tmp.as<float>();
    va.g_out = s->tmp.as<float>() + VN;
    va.g_transposed = 0;
    batch_rows(s, va);
    HIPCHK(launch_var(va, VOP_GRAD, var_blocks(s, va.V), s->stream));
    if (U) HIPCHK(hipMemcpyAsync(U, va.U_out, VN * 4, hipMemcpyDeviceToHost, s->stream));
    if (g) HIPCHK(hipMemcpyAsync(g, va.g_out, VN * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

int32_t tsat_extract_partial(tsat_solver* s, int32_t max_cands, int32_t k, int32_t* cand_ids, int32_t* lits,
                             int64_t* sat_counts)
{
    g_err.clear();
    RET(need_batch(s));
    RET(need_single(s));
    if (s->rows_per_var == 2) return fail(TSAT_E_STATE, "the hand-off buffer takes complete assignments (literal rows are on)");
    if (max_cands < 1 || max_cands > s->N) return fail(TSAT_E_ARG, "max_cands must be in [1, %d]", s->N);
    if (k <= 0) k = s->params.k_partial;
    if (k <= 0) k = (int32_t)std::max<int64_t>(20, ((int64_t)s->st.V + 9999) / 10000);
    if (k > 4096) return fail(TSAT_E_ARG, "k must be <= 4096 (got %d)", k);
    if (!cand_ids || !lits) return fail(TSAT_E_ARG, "NULL output");
    RET(ensure_mode(s, s->params.norm_mode));
    RET(ensure_scratch(s, s->N));
    const size_t VN = (size_t)s->st.V * s->N;
    DBuf gT, order, lout, cout;
    RET(gT.alloc(VN * 4, "transposed gradient"));
    RET(order.alloc((size_t)s->N * 4, "candidate order"));
    RET(lout.alloc((size_t)max_cands * k * 4, "partial assignments"));
    RET(cout.alloc((size_t)max_cands * 4, "candidate ids"));
    RET(eval_rows(s, s->params, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, nullptr, nullptr, nullptr,
                  s->sat_scr.as<int64_t>(), s->table_scr.as<float>(), s->stream));
    VarArgs va = var_args(s, s->params, s->N, s->W, s->Np);
    va.tbl = s->table_scr.as<float>();
    va.theta = s->theta.as<float>();
    va.lits_cur = s->lits[s->cur].as<uint64_t>();
    va.mu_cur = s->mu[s->cur].as<double>();
    va.g_out = gT.as<float>();
    va.g_transposed = 1;
    HIPCHK(launch_var(va, VOP_GRAD, var_blocks(s, s->st.V), s->stream));
    HIPCHK(launch_rank(s->sat_scr.as<int64_t>(), s->N, order.as<int32_t>(), s->stream));
    SelectArgs sa{};
    sa.gT = gT.as<float>();
    sa.occ_off = s->occ_off.as<uint32_t>();
    sa.lits = s->lits[s->cur].as<uint64_t>();
    sa.order = order.as<int32_t>();
    sa.V = s->st.V;
    sa.W = s->W;
    sa.k = k;
    int kp = 1;
    while (kp < k) kp <<= 1;
    sa.kpow2 = kp;
    sa.lits_out = lout.as<int32_t>();
    sa.cand_out = cout.as<int32_t>();
    HIPCHK(launch_select(sa, max_cands, s->stream));
    std::vector<int64_t> sat(s->N);
    HIPCHK(hipMemcpyAsync(lits, lout.p, (size_t)max_cands * k * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(cand_ids, cout.p, (size_t)max_cands * 4, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(sat.data(), s->sat_scr.p, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (sat_counts)
        for (int32_t a = 0; a < max_cands; ++a) sat_counts[a] = sat[cand_ids[a]];
    return TSAT_OK;
}

// ------------------------------------------------------- device-pointer API

int32_t tsat_pack_dev(tsat_solver* s, const float* assign, int32_t N, uint64_t* bits, void* stream)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || !assign || !bits) return fail(TSAT_E_ARG, "invalid arguments");
    RET(set_dev(s));
    hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    HIPCHK(launch_pack(assign, s->st.V, N, (N + 63) / 64, bits, 0, st));
    return TSAT_OK;
}

static int32_t dev_prepare(tsat_solver* s, const uint64_t* bits, int32_t N, hipStream_t st)
{
    RET(need_single(s));
    RET(ensure_scratch(s, N));
    RET(prepare_units(s, N));
    HIPCHK(launch_expand(bits, s->st.V, (N + 63) / 64, N, s->lits_scr.as<uint64_t>(), st));
    return TSAT_OK;
}

int32_t tsat_fwd_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, float* S, uint32_t* hist, void* stream)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || !bits || !(tau >= 0.f)) return fail(TSAT_E_ARG, "invalid arguments");
    RET(set_dev(s));
    hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    RET(dev_prepare(s, bits, N, st));
    tsat_params p = s->params;
    p.tau = tau;
    return eval_rows(s, p, s->lits_scr.as<uint64_t>(), N, nullptr, hist, S, nullptr, nullptr, nullptr, st);
}

int32_t tsat_bwd_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, const float* dS, float* U, void* stream)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || N > TSAT_MAX_STEP_N || !bits || !dS || !U || !(tau >= 0.f)) return fail(TSAT_E_ARG, "invalid arguments");
    RET(set_dev(s));
    hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    if ((size_t)K1_of(s) * Np * 4 > 64 * 1024) return fail(TSAT_E_ARG, "table exceeds 64 KiB");
    RET(check_row_offsets(s, W));
    RET(dev_prepare(s, bits, N, st));
    tsat_params p = s->params;
    p.tau = tau;
    RET(eval_rows(s, p, s->lits_scr.as<uint64_t>(), N, dS, nullptr, nullptr, nullptr, nullptr, s->table_scr.as<float>(), st));
    VarArgs va = var_args(s, p, N, W, Np);
    va.tbl = s->table_scr.as<float>();
    va.lits_cur = s->lits_scr.as<uint64_t>();
    va.U_out = U;
    HIPCHK(launch_var(va, VOP_ADJ, var_blocks(s, s->st.V), st));
    return TSAT_OK;
}

int32_t tsat_bwd_scatter_dev(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, const float* dS, float* U,
                             void* stream)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || N > 256 || !bits || !dS || !U || !(tau >= 0.f)) return fail(TSAT_E_ARG, "invalid arguments");
    RET(set_dev(s));
    hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    if ((size_t)K1_of(s) * Np * 4 > 48 * 1024) return fail(TSAT_E_ARG, "table exceeds 48 KiB");
    RET(dev_prepare(s, bits, N, st));
    tsat_params p = s->params;
    p.tau = tau;
    RET(eval_rows(s, p, s->lits_scr.as<uint64_t>(), N, dS, nullptr, nullptr, nullptr, nullptr, s->table_scr.as<float>(), st));
    HIPCHK(launch_fill_u32(reinterpret_cast<uint32_t*>(U), (int64_t)s->st.V * N, 0u, st));
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0) continue;
        HIPCHK(launch_adj_scatter(b->codes.as<uint32_t>(), b->count, b->k, N, K1_of(s),
                                  reinterpret_cast<const uint32_t*>(s->lits_scr.p), 2 * W, s->table_scr.as<float>(), U,
                                  s->st.V, st));
    }
    return TSAT_OK;
}

int32_t tsat_fwd_dev_noalloc(tsat_solver* s, const uint64_t* bits, int32_t N, float tau, float* S, uint32_t* hist,
                             void* stream)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || N > TSAT_MAX_STEP_N || !bits || !(tau >= 0.f) || !std::isfinite(tau))
        return fail(TSAT_E_ARG, "invalid arguments");
    RET(need_single(s));
    if (!s->noalloc_scratch) return fail(TSAT_E_HIP, "scratch array address unavailable (HIP error %d)", s->noalloc_rc);
    RET(set_dev(s));
    hipStream_t st = (hipStream_t)stream; // NULL: the null (default) stream
    const int32_t W = (N + 63) / 64, Np = 64 * W, K1 = K1_of(s);
    // layout: histogram accumulator [Np][K1] u32, then each bucket's units
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t h_bytes = up((size_t)Np * K1 * 4);
    size_t need = h_bytes;
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0) continue;
        const FwdGeom g = fwd_geometry(N, K1, b->count, b->k, s->fwd_target_blocks);
        const int64_t per = (int64_t)g.S * g.CPT;
        need += up((size_t)((b->count + per - 1) / per) * sizeof(FwdUnit));
    }
    if (need > TSAT_NOALLOC_SCRATCH_BYTES)
        return fail(TSAT_E_ARG, "needs %zu bytes of scratch, the fixed array holds %u", need, TSAT_NOALLOC_SCRATCH_BYTES);
    uint8_t* base = static_cast<uint8_t*>(s->noalloc_scratch);
    uint32_t* H = reinterpret_cast<uint32_t*>(base);
    HIPCHK(launch_fill_u32(H, (int64_t)Np * K1, 0u, st));
    size_t off = h_bytes;
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0) continue;
        const FwdGeom g = fwd_geometry(N, K1, b->count, b->k, s->fwd_target_blocks);
        const int64_t per = (int64_t)g.S * g.CPT;
        const int64_t nunits = (b->count + per - 1) / per;
        FwdUnit* units = reinterpret_cast<FwdUnit*>(base + off);
        off += up((size_t)nunits * sizeof(FwdUnit));
        HIPCHK(launch_fwd_units(units, nunits, per, b->count, st));
        FwdArgs a{};
        a.units = units;
        a.codes = b->codes.as<uint32_t>();
        a.KW = b->k;
        a.K1 = K1;
        a.bits32 = reinterpret_cast<const uint32_t*>(bits);
        a.W2 = 2 * W;
        a.vrows = 1;
        a.Dn = g.Dn;
        a.DT = g.DT;
        a.CPT = g.CPT;
        a.H = H;
        a.H_stride = (int64_t)Np * K1;
        a.nunits = (int32_t)nunits;
        HIPCHK(launch_fwd(a, (int)nunits, g.tiles, st));
    }
    tsat_params p = s->params;
    p.tau = tau;
    SminArgs a = smin_args(s, p, N, Np);
    a.H = H;
    a.H_last = hist;
    a.S_out = S;
    a.update = 0;
    HIPCHK(launch_smin(a, st));
    return TSAT_OK;
}

// Eq. 5 + Eq. 2 of caller logits into the scratch literal rows (and row
// means), optionally also the value rows and 0/1 floats for the caller.
static int32_t dev_binarize(tsat_solver* s, const float* theta, int32_t N, int32_t mode, uint64_t* vbits, float* assign,
                            double* mu, hipStream_t st)
{
    RET(need_single(s));
    RET(ensure_scratch(s, N));
    RET(prepare_units(s, N));
    const int32_t W = (N + 63) / 64;
    tsat_params p = s->params;
    p.norm_mode = mode;
    VarArgs a = var_args(s, p, N, W, 64 * W);
    a.theta = const_cast<float*>(theta); // read only by the binarize op
    a.lits_next = s->lits_scr.as<uint64_t>();
    a.mu_next = mu ? mu : s->mu_scr.as<double>();
    a.vbits_out = vbits;
    a.assign_out = assign;
    HIPCHK(launch_var(a, VOP_BINARIZE, var_blocks(s, s->st.V), st));
    return TSAT_OK;
}

static int32_t dev_args(tsat_solver* s, int32_t N, int32_t mode, const void* theta, float tau)
{
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || N > TSAT_MAX_STEP_N) return fail(TSAT_E_ARG, "N must be in [1, %d]", TSAT_MAX_STEP_N);
    if (mode != TSAT_MODE_MEAN && mode != TSAT_MODE_NONE) return fail(TSAT_E_ARG, "mode must be 0 or 1");
    if (!theta) return fail(TSAT_E_ARG, "theta is NULL");
    if (!(tau >= 0.f) || !std::isfinite(tau)) return fail(TSAT_E_ARG, "tau must be finite and >= 0");
    return set_dev(s);
}

int32_t tsat_binarize_dev(tsat_solver* s, const float* theta, int32_t N, int32_t mode, uint64_t* bits, float* assign,
                          double* mu, void* stream)
{
    g_err.clear();
    RET(dev_args(s, N, mode, theta, 0.f));
    if (!bits && !assign && !mu) return fail(TSAT_E_ARG, "no output");
    RET(check_row_offsets(s, (N + 63) / 64));
    return dev_binarize(s, theta, N, mode, bits, assign, mu, (hipStream_t)stream);
}

int32_t tsat_norm_backward_dev(tsat_solver* s, const float* theta, const float* dA, int32_t N, int32_t mode, float* g,
                               void* stream)
{
    g_err.clear();
    RET(dev_args(s, N, mode, theta, 0.f));
    if (!dA || !g) return fail(TSAT_E_ARG, "NULL dA or g");
    const int32_t W = (N + 63) / 64;
    tsat_params p = s->params;
    p.norm_mode = mode;
    VarArgs a = var_args(s, p, N, W, 64 * W);
    a.theta = const_cast<float*>(theta); // read only by this op
    a.dA_in = dA;
    a.g_out = g;
    HIPCHK(launch_var(a, VOP_NORMBWD, var_blocks(s, s->st.V), (hipStream_t)stream));
    return TSAT_OK;
}

int32_t tsat_loss_dev(tsat_solver* s, const float* theta, int32_t N, float tau, int32_t mode, float* loss, float* S,
                      uint64_t* bits, void* stream)
{
    g_err.clear();
    RET(dev_args(s, N, mode, theta, tau));
    if (!loss) return fail(TSAT_E_ARG, "loss is NULL");
    RET(check_row_offsets(s, (N + 63) / 64));
    hipStream_t st = (hipStream_t)stream;
    RET(dev_binarize(s, theta, N, mode, bits, nullptr, nullptr, st));
    tsat_params p = s->params;
    p.tau = tau;
    p.norm_mode = mode;
    return eval_rows(s, p, s->lits_scr.as<uint64_t>(), N, nullptr, nullptr, S, nullptr, nullptr, nullptr, st, loss);
}

int32_t tsat_loss_backward_dev(tsat_solver* s, const float* theta, int32_t N, float tau, int32_t mode,
                               const float* dloss, float* g, float* U, void* stream)
{
    g_err.clear();
    RET(dev_args(s, N, mode, theta, tau));
    if (!g) return fail(TSAT_E_ARG, "g is NULL");
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    if ((size_t)K1_of(s) * Np * 4 > 64 * 1024) return fail(TSAT_E_ARG, "table exceeds 64 KiB");
    RET(check_row_offsets(s, W));
    hipStream_t st = (hipStream_t)stream;
    RET(dev_binarize(s, theta, N, mode, nullptr, nullptr, nullptr, st));
    tsat_params p = s->params;
    p.tau = tau;
    p.norm_mode = mode;
    RET(eval_rows(s, p, s->lits_scr.as<uint64_t>(), N, nullptr, nullptr, nullptr, nullptr, nullptr,
                  s->table_scr.as<float>(), st, nullptr, dloss));
    VarArgs va = var_args(s, p, N, W, Np);
    va.tbl = s->table_scr.as<float>();
    va.theta = const_cast<float*>(theta); // read only by the gradient op
    va.lits_cur = s->lits_scr.as<uint64_t>();
    va.mu_cur = s->mu_scr.as<double>();
    va.U_out = U;
    va.g_out = g;
    va.g_transposed = 0;
    HIPCHK(launch_var(va, VOP_GRAD, var_blocks(s, s->st.V), st));
    return TSAT_OK;
}

// ------------------------------------------------------------------ timing

static int32_t check_launch_config(const tsat_launch_config* c)
{
    if (c->fwd_target_blocks < 1 || c->fwd_target_blocks > (1 << 20))
        return fail(TSAT_E_ARG, "fwd_target_blocks must be in [1, 2^20]");
    if (c->var_blocks_per_cu < 0 || c->var_blocks_per_cu > 1024)
        return fail(TSAT_E_ARG, "var_blocks_per_cu must be in [0, 1024]");
    if (c->pure_group != 1 && c->pure_group != 2 && c->pure_group != 4)
        return fail(TSAT_E_ARG, "pure_group must be 1, 2 or 4");
    if (c->clause_planes != 0 && c->clause_planes != 1) return fail(TSAT_E_ARG, "clause_planes must be 0 or 1");
    if (c->window_gather != 0 && c->window_gather != 1) return fail(TSAT_E_ARG, "window_gather must be 0 or 1");
    return TSAT_OK;
}

int32_t tsat_get_launch_config(tsat_solver* s, tsat_launch_config* out)
{
    g_err.clear();
    if (!s || !out) return fail(TSAT_E_ARG, "NULL argument");
    memset(out, 0, sizeof *out);
    out->fwd_target_blocks = s->fwd_target_blocks;
    out->var_blocks_per_cu = s->var_per_cu;
    out->pure_group = s->pure_group;
    out->clause_planes = s->clause_planes;
    out->window_gather = s->window_gather;
    return TSAT_OK;
}

int32_t tsat_set_launch_config(tsat_solver* s, const tsat_launch_config* cfg)
{
    g_err.clear();
    if (!s || !cfg) return fail(TSAT_E_ARG, "NULL argument");
    RET(check_launch_config(cfg));
    if (s->rows_per_var == 2 && s->N > 0 && (!cfg->clause_planes || !cfg->window_gather))
        return fail(TSAT_E_ARG, "independent literal rows need the clause planes and the window gather");
    RET(set_dev(s));
    HIPCHK(hipStreamSynchronize(s->stream));
    s->drop_graph();
    s->fwd_target_blocks = cfg->fwd_target_blocks;
    s->var_per_cu = cfg->var_blocks_per_cu;
    s->pure_group = cfg->pure_group;
    s->clause_planes = cfg->clause_planes;
    s->window_gather = cfg->window_gather;
    if (s->N > 0 && plane_path(s, s->N)) RET(ensure_planes(s, s->planes, s->N, s->stream));
    return TSAT_OK;
}

// Time `iters` eager iterations under the current launch shape; per-kernel
// averages (forward, SmoothMin, fused update) in ms.
static int32_t time_iterations(tsat_solver* s, int32_t iters, const tsat_params* p, double ms[3])
{
    const bool timing = s->timing, graph = s->use_graph;
    s->timing = true;
    s->use_graph = false;
    tsat_report rep;
    const int32_t rc = tsat_step(s, iters, p, 0, &rep);
    s->timing = timing;
    s->use_graph = graph;
    if (rc != TSAT_OK) return rc;
    if (s->timed_iters == 0) return fail(TSAT_E_STATE, "no timed iterations");
    for (int k = 0; k < 3; ++k) ms[k] = s->timed_ms[k];
    return TSAT_OK;
}

int32_t tsat_autotune(tsat_solver* s, int32_t iters, const tsat_params* p, tsat_launch_config* best,
                      int32_t* iters_used)
{
    g_err.clear();
    RET(need_batch(s));
    if (iters < 1 || iters > 64) return fail(TSAT_E_ARG, "iters must be in [1, 64]");
    int32_t used = 0;
    double ms[3];
    tsat_launch_config cur;
    RET(tsat_get_launch_config(s, &cur));
    // forward work-unit target: only the forward kernels depend on it.  What
    // counts is the clauses per thread that follow from it (a short loop
    // leaves latency exposed, a long one spreads an XCD's resident blocks
    // over too many rows for its L2), so large batches need large targets
    static const int kFwd[] = {256, 512, 1024, 2048, 4096, 8192, 16384, 32768};
    double best_fwd = 1e30;
    int pick_fwd = cur.fwd_target_blocks;
    for (int f : kFwd) {
        tsat_launch_config c = cur;
        c.fwd_target_blocks = f;
        RET(tsat_set_launch_config(s, &c));
        RET(prepare_units(s, s->N));
        RET(time_iterations(s, iters, p, ms));
        used += iters;
        if (ms[0] < best_fwd) {
            best_fwd = ms[0];
            pick_fwd = f;
        }
    }
    cur.fwd_target_blocks = pick_fwd;
    // fused update kernel: blocks per CU, and the record grouping of
    // uniform-width stores
    // (a large ragged batch runs best far beyond the resident blocks: waves
    // then take few chunks each, and the chip walks the variables in order)
    static const int kPerCu[] = {0, 8, 16, 32, 64, 128, 256, 512, 1024};
    const bool pure = s->st.pure_k != 0;
    const bool planes_apply = s->occ_cid.p && (s->N + 63) / 64 <= 4;
    static const int kGroups[] = {1, 2, 4};
    double best_var = 1e30, best_sum = 1e30;
    tsat_launch_config pick = cur;
    // with clause planes the record group does not apply (the planes come in
    // by 64-record windows or record by record); the forward writes the
    // planes, so the shapes are compared on forward + update time
    for (int cp = planes_apply ? 1 : 0; cp >= (s->rows_per_var == 2 ? 1 : 0); --cp) {
        const int ngroups = (pure && !cp) ? 3 : 1;
        const int nwin = (cp && uniform_plane_store(s) && s->rows_per_var == 1) ? 2 : 1;
        for (int pc : kPerCu) {
            for (int gi = 0; gi < ngroups; ++gi) {
                for (int wi = 0; wi < nwin; ++wi) {
                    tsat_launch_config c = cur;
                    c.var_blocks_per_cu = pc;
                    c.pure_group = ngroups > 1 ? kGroups[gi] : cur.pure_group;
                    c.clause_planes = planes_apply ? cp : cur.clause_planes;
                    c.window_gather = nwin > 1 ? 1 - wi : (cp ? 1 : cur.window_gather);
                    RET(tsat_set_launch_config(s, &c));
                    RET(time_iterations(s, iters, p, ms));
                    used += iters;
                    if (ms[0] + ms[2] < best_sum) {
                        best_sum = ms[0] + ms[2];
                        best_var = ms[2];
                        best_fwd = ms[0];
                        pick = c;
                    }
                }
            }
        }
    }
    RET(tsat_set_launch_config(s, &pick));
    if (best) {
        *best = pick;
        best->fwd_ms = best_fwd;
        best->var_ms = best_var;
    }
    if (iters_used) *iters_used = used;
    return TSAT_OK;
}

int32_t tsat_set_timing(tsat_solver* s, int32_t enable)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    s->timing = enable != 0;
    return TSAT_OK;
}

int32_t tsat_get_timing(tsat_solver* s, double* ms, int32_t* iters)
{
    g_err.clear();
    if (!s || !ms) return fail(TSAT_E_ARG, "NULL argument");
    if (s->timed_iters == 0) return fail(TSAT_E_STATE, "no timed iterations");
    for (int k = 0; k < 3; ++k) ms[k] = s->timed_ms[k];
    if (iters) *iters = s->timed_iters;
    return TSAT_OK;
}

int32_t tsat_copy_calibrate(tsat_solver* s, int64_t bytes, double* ms)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (bytes < 16 || bytes % 16) return fail(TSAT_E_ARG, "bytes must be a positive multiple of 16");
    RET(set_dev(s));
    DBuf a, b;
    RET(a.alloc((size_t)bytes, "copy source"));
    RET(b.alloc((size_t)bytes, "copy destination"));
    HIPCHK(launch_fill_u32(a.as<uint32_t>(), bytes / 4, 1u, s->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TSAT_E_HIP, "hipEventCreate failed");
    }
    hipError_t err = hipEventRecord(e0, s->stream);
    if (err == hipSuccess) err = launch_copy16(b.p, a.p, bytes / 16, 8 * s->cus, s->stream);
    if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(TSAT_E_HIP, "copy kernel failed: %s", hipGetErrorString(err));
    if (ms) *ms = t;
    return TSAT_OK;
}

int32_t tsat_set_literal_rows(tsat_solver* s, int32_t enable)
{
    g_err.clear();
    RET(need_loaded(s));
    if (enable != 0 && enable != 1) return fail(TSAT_E_ARG, "enable must be 0 or 1");
    HIPCHK(hipStreamSynchronize(s->stream));
    if (enable) {
        RET(need_single(s));
        if (!s->occ_cid.p) return fail(TSAT_E_ARG, "independent literal rows need clauses at most %d wide", kMaxPlaneWidth);
        if (s->st.max_sign_rec >= 65536) return fail(TSAT_E_ARG, "a literal occurs in 65536 or more clauses");
        // literal l = 2 v + neg owns the records [lro[l], lro[l + 1]): the
        // variable's positive records, then its negative ones
        const std::vector<uint32_t>& off = s->st.cid_off.empty() ? s->st.occ_off : s->st.cid_off;
        const std::vector<uint32_t>& mid = s->st.cid_off.empty() ? s->st.occ_mid : s->st.cid_mid;
        const size_t V = (size_t)s->st.V;
        std::vector<uint32_t> lro;
        try {
            lro.resize(2 * V + 1);
        } catch (const std::bad_alloc&) {
            return fail(TSAT_E_OOM, "host allocation failed");
        }
        for (size_t v = 0; v < V; ++v) {
            lro[2 * v] = off[v];
            lro[2 * v + 1] = mid[v];
        }
        lro[2 * V] = off[V];
        RET(s->lro.alloc((2 * V + 1) * 4, "literal record offsets"));
        HIPCHK(hipMemcpy(s->lro.p, lro.data(), (2 * V + 1) * 4, hipMemcpyHostToDevice));
    }
    s->lit_rows_req = enable;
    // the layout changes with the next batch; the current one is dropped
    s->drop_graph();
    s->N = 0;
    return TSAT_OK;
}

int32_t tsat_stream_calibrate(tsat_solver* s, int64_t bytes, int32_t kind, int32_t reps, double* ms)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (bytes < 16384 || bytes % 16384) return fail(TSAT_E_ARG, "bytes must be a positive multiple of 16384");
    if (kind < 0 || kind > 2) return fail(TSAT_E_ARG, "kind must be 0, 1 or 2");
    if (reps < 1 || reps > 1000) return fail(TSAT_E_ARG, "reps must be in [1, 1000]");
    RET(set_dev(s));
    DBuf a, b, c, src;
    RET(a.alloc((size_t)bytes, "stream array"));
    if (kind == 0) {
        RET(src.alloc((size_t)bytes, "stream source"));
        HIPCHK(launch_fill_u32(src.as<uint32_t>(), bytes / 4, 1u, s->stream));
    } else {
        RET(b.alloc((size_t)bytes, "stream array"));
        RET(c.alloc((size_t)bytes, "stream array"));
        HIPCHK(launch_fill_u32(b.as<uint32_t>(), bytes / 4, 2u, s->stream));
        HIPCHK(launch_fill_u32(c.as<uint32_t>(), bytes / 4, 3u, s->stream));
    }
    HIPCHK(launch_fill_u32(a.as<uint32_t>(), bytes / 4, 1u, s->stream));
    const int64_t n4 = bytes / 16;
    // every block a few passes over its share: 8 blocks per CU
    const int blocks = 8 * s->cus;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(TSAT_E_HIP, "hipEventCreate failed");
    }
    // one untimed launch, then reps timed ones
    hipError_t err = launch_stream(kind, a.as<uint32_t>(), b.as<uint32_t>(), c.as<uint32_t>(), src.as<uint32_t>(), n4,
                                   blocks, s->stream);
    if (err == hipSuccess) err = hipEventRecord(e0, s->stream);
    for (int32_t r = 0; r < reps && err == hipSuccess; ++r)
        err = launch_stream(kind, a.as<uint32_t>(), b.as<uint32_t>(), c.as<uint32_t>(), src.as<uint32_t>(), n4, blocks,
                            s->stream);
    if (err == hipSuccess) err = hipEventRecord(e1, s->stream);
    if (err == hipSuccess) err = hipEventSynchronize(e1);
    float t = 0.f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(TSAT_E_HIP, "stream kernel failed: %s", hipGetErrorString(err));
    if (ms) *ms = t / reps;
    return TSAT_OK;
}

} // extern "C"
