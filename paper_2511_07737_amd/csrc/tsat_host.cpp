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
#include <new>
#include <string>
#include <vector>

#include "tsat.h"
#include "tsat_device.h"

using namespace tsat;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_err;

static int32_t fail(int32_t code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(x)                                                                            \
    do {                                                                                     \
        hipError_t e_ = (x);                                                                 \
        if (e_ != hipSuccess) return fail(TSAT_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)

#define RET(x)                       \
    do {                             \
        int32_t r_ = (x);            \
        if (r_ != TSAT_OK) return r_; \
    } while (0)

// allocation-failure injection for tests of the OOM path
static int64_t g_fail_alloc_countdown = -2;

static bool inject_alloc_failure()
{
    if (g_fail_alloc_countdown == -2) {
        const char* e = getenv("TSAT_FAIL_ALLOC_AFTER");
        g_fail_alloc_countdown = e ? atoll(e) : -1;
    }
    if (g_fail_alloc_countdown < 0) return false;
    if (g_fail_alloc_countdown == 0) return true;
    --g_fail_alloc_countdown;
    return false;
}

// ---------------------------------------------------------------------------
// device buffers
// ---------------------------------------------------------------------------

struct DBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DBuf() = default;
    DBuf(const DBuf&) = delete;
    DBuf& operator=(const DBuf&) = delete;
    ~DBuf() { release(); }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    int32_t alloc(size_t n, const char* what)
    {
        if (n == bytes && p) return TSAT_OK;
        release();
        if (n == 0) return TSAT_OK;
        if (inject_alloc_failure()) return fail(TSAT_E_OOM, "device allocation of %zu bytes for %s failed (injected)", n, what);
        if (hipMalloc(&p, n) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            return fail(TSAT_E_OOM, "device allocation of %zu bytes for %s failed", n, what);
        }
        bytes = n;
        return TSAT_OK;
    }
    // grow-only variant for scratch space
    int32_t reserve(size_t n, const char* what) { return (n <= bytes && p) ? TSAT_OK : alloc(n, what); }
    template <class T> T* as() const { return static_cast<T*>(p); }
};

// ---------------------------------------------------------------------------
// host-side clause store (Sec. III-A; sparse P of Sec. IV-A)
// ---------------------------------------------------------------------------

struct Store {
    int32_t V = 0;
    int32_t K = 0;       // widest clause
    int64_t C = 0;       // clauses including empty ones
    int64_t L = 0;       // literal occurrences
    int64_t n_empty = 0;
    int64_t n_dup = 0;
    int64_t n_taut = 0;
    int64_t width_count[TSAT_MAX_WIDTH + 1] = {0};
    std::vector<std::vector<uint32_t>> buckets; // [k] -> [Cb][k] literal codes 2*var+neg
    // occurrence store with literal codes (converted to byte offsets on upload)
    std::vector<uint32_t> occ_off, occ_mid, occ_data;
};

static inline uint32_t lit_code(int32_t x) { return x > 0 ? 2u * (uint32_t)(x - 1) : 2u * (uint32_t)(-x - 1) + 1u; }

static int32_t build_store(int32_t V, int64_t n, const int32_t* lits, Store& st, bool with_occ)
{
    if (V < 1) return fail(TSAT_E_ARG, "num_vars must be >= 1 (got %d)", V);
    if (n < 0 || (n > 0 && !lits)) return fail(TSAT_E_ARG, "invalid literal stream (n=%lld)", (long long)n);
    if (n > 0 && lits[n - 1] != 0) return fail(TSAT_E_ARG, "the last clause is not terminated by 0");
    if ((int64_t)2 * V > (int64_t)0x7fffffff) return fail(TSAT_E_ARG, "too many variables (%d)", V);
    st = Store();
    st.V = V;
    std::vector<uint32_t> cl;
    std::vector<std::vector<uint32_t>> buckets(TSAT_MAX_WIDTH + 1);
    int64_t start = 0;
    try {
        for (int64_t j = 0; j < n; ++j) {
            const int32_t x = lits[j];
            if (x != 0) {
                const int64_t a = x < 0 ? -(int64_t)x : (int64_t)x;
                if (a > V) return fail(TSAT_E_ARG, "literal %d at position %lld exceeds num_vars=%d", x, (long long)j, V);
                continue;
            }
            cl.clear();
            for (int64_t q = start; q < j; ++q) cl.push_back(lit_code(lits[q]));
            start = j + 1;
            std::sort(cl.begin(), cl.end());
            const size_t before = cl.size();
            cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
            st.n_dup += (int64_t)(before - cl.size());
            for (size_t q = 1; q < cl.size(); ++q)
                if ((cl[q] >> 1) == (cl[q - 1] >> 1)) { ++st.n_taut; break; }
            const size_t k = cl.size();
            if (k > TSAT_MAX_WIDTH)
                return fail(TSAT_E_ARG, "clause %lld has %zu distinct literals (max %d)", (long long)st.C, k, TSAT_MAX_WIDTH);
            buckets[k].insert(buckets[k].end(), cl.begin(), cl.end());
            st.width_count[k] += 1;
            if ((int)k > st.K) st.K = (int)k;
            st.C += 1;
            st.L += (int64_t)k;
        }
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed while building the clause store");
    }
    st.n_empty = st.width_count[0];
    st.buckets = std::move(buckets);
    if (!with_occ) return TSAT_OK;
    // per variable: records of positive occurrences, then negative ones;
    // record = (k-1, codes of the other k-1 literals)
    try {
        std::vector<uint64_t> wpos(V, 0), wneg(V, 0);
        for (int k = 1; k <= st.K; ++k) {
            const auto& b = st.buckets[k];
            for (size_t q = 0; q < b.size(); ++q) {
                const uint32_t c = b[q];
                (c & 1u ? wneg : wpos)[c >> 1] += (uint64_t)k;
            }
        }
        uint64_t total = 0;
        st.occ_off.assign((size_t)V + 1, 0);
        st.occ_mid.assign((size_t)V, 0);
        for (int32_t v = 0; v < V; ++v) {
            st.occ_off[v] = (uint32_t)total;
            st.occ_mid[v] = (uint32_t)(total + wpos[v]);
            total += wpos[v] + wneg[v];
            if (total > 0xffffffffull) return fail(TSAT_E_ARG, "occurrence store exceeds 2^32 words");
        }
        st.occ_off[V] = (uint32_t)total;
        st.occ_data.assign(total, 0);
        std::vector<uint32_t> curp(V), curn(V);
        for (int32_t v = 0; v < V; ++v) {
            curp[v] = st.occ_off[v];
            curn[v] = st.occ_mid[v];
        }
        for (int k = 1; k <= st.K; ++k) {
            const auto& b = st.buckets[k];
            const size_t Cb = b.size() / (size_t)k;
            for (size_t c = 0; c < Cb; ++c) {
                const uint32_t* lit = &b[c * k];
                for (int e = 0; e < k; ++e) {
                    const uint32_t code = lit[e];
                    uint32_t& pos = (code & 1u) ? curn[code >> 1] : curp[code >> 1];
                    st.occ_data[pos++] = (uint32_t)(k - 1);
                    for (int f = 0; f < k; ++f)
                        if (f != e) st.occ_data[pos++] = lit[f];
                }
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed while building the occurrence store");
    }
    return TSAT_OK;
}

// ---------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------

struct Bucket {
    int32_t k;
    int64_t count;
    DBuf codes;
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
    DBuf occ_off, occ_mid, occ_data;

    // batch
    int32_t N = 0, W = 0, Np = 0;
    DBuf lits[2];
    int cur = 0;
    int32_t bits_mode = TSAT_MODE_MEAN; // normalization mode the current bits were computed with
    DBuf theta, m, v;
    DBuf H, H_last, table, S64, sat;
    DBuf ctrl, ctrl_scr, witness;
    // scratch for stateless evaluations and the device-pointer API
    DBuf lits_scr, H_scr, table_scr, S64_scr, sat_scr, tmp;
    int32_t scr_Np = 0;

    // timing
    bool timing = false;
    std::vector<hipEvent_t> events;
    double timed_ms[3] = {0, 0, 0};
    int32_t timed_iters = 0;

    ~tsat_solver()
    {
        for (auto* b : buckets) delete b;
        for (auto e : events) (void)hipEventDestroy(e);
        if (own_stream && stream) (void)hipStreamDestroy(stream);
    }
};

static int32_t K1_of(const tsat_solver* s) { return s->st.K + 1; }

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
    return TSAT_OK;
}

// launch geometry of the forward pass for one width bucket
static void fwd_geometry(int32_t W2, int32_t K1, int64_t Cb, int32_t KW, int32_t& DT, int32_t& CPT, dim3& grid)
{
    int bins = (KW <= 4) ? KW + 1 : K1;
    DT = std::min(W2, 64);
    while (DT > 1 && (size_t)DT * 32 * bins * 4 > 64 * 1024) DT >>= 1;
    const int S = 256 / DT;
    const int gy = (W2 + DT - 1) / DT;
    const int64_t target_x = std::max<int64_t>(1, (2048 + gy - 1) / gy);
    int64_t cpt = (Cb + (int64_t)S * target_x - 1) / ((int64_t)S * target_x);
    cpt = std::max<int64_t>(16, std::min<int64_t>(255, cpt));
    CPT = (int32_t)cpt;
    const int64_t gx = (Cb + (int64_t)S * cpt - 1) / ((int64_t)S * cpt);
    grid = dim3((unsigned)std::max<int64_t>(1, gx), (unsigned)gy, 1);
}

// enqueue the forward histogram of every width bucket on literal rows `lits`
static int32_t enqueue_fwd(tsat_solver* s, const uint64_t* lits, int32_t W, uint32_t* H, const Ctrl* ctrl, hipStream_t st)
{
    for (auto* b : s->buckets) {
        if (b->count == 0 || b->k == 0) continue;
        FwdArgs a{};
        a.codes = b->codes.as<uint32_t>();
        a.Cb = b->count;
        a.KW = b->k;
        a.K1 = K1_of(s);
        a.bits32 = reinterpret_cast<const uint32_t*>(lits);
        a.W2 = 2 * W;
        a.H = H;
        a.ctrl = ctrl;
        dim3 grid;
        fwd_geometry(a.W2, a.K1, a.Cb, a.KW, a.DT, a.CPT, grid);
        HIPCHK(launch_fwd(a, grid, st));
    }
    return TSAT_OK;
}

static SminArgs smin_args(tsat_solver* s, const tsat_params& p, int32_t N, int32_t Np)
{
    SminArgs a{};
    a.C = s->st.C;
    a.n_empty = s->st.n_empty;
    a.N = N;
    a.Np = Np;
    a.K1 = K1_of(s);
    a.zero_H = 1;
    a.every = p.decay_every;
    a.restart = p.restart_every;
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

static int var_blocks(const tsat_solver* s, int32_t V)
{
    const int64_t want = ((int64_t)V + 3) / 4;
    return (int)std::max<int64_t>(1, std::min<int64_t>(want, (int64_t)s->cus * 8));
}

static VarArgs var_args(tsat_solver* s, const tsat_params& p, int32_t N, int32_t W, int32_t Np)
{
    VarArgs a{};
    a.V = s->st.V;
    a.N = N;
    a.W = W;
    a.Np = Np;
    a.K1 = K1_of(s);
    a.mode = p.norm_mode;
    a.occ_off = s->occ_off.as<uint32_t>();
    a.occ_mid = s->occ_mid.as<uint32_t>();
    a.occ_data = s->occ_data.as<uint32_t>();
    a.beta1 = (float)p.beta1;
    a.beta2 = (float)p.beta2;
    a.one_minus_beta1 = (float)(1.0 - p.beta1);
    a.one_minus_beta2 = (float)(1.0 - p.beta2);
    a.eps = (float)p.eps;
    return a;
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
    RET(s->lits_scr.reserve((size_t)2 * s->st.V * W * 8, "scratch literal rows"));
    if (Np > s->scr_Np) {
        RET(s->H_scr.alloc((size_t)Np * K1 * 4, "scratch histogram"));
        HIPCHK(launch_fill_u32(s->H_scr.as<uint32_t>(), (int64_t)Np * K1, 0u, s->stream));
        RET(s->table_scr.alloc((size_t)Np * K1 * 4, "scratch table"));
        RET(s->S64_scr.alloc((size_t)Np * 8, "scratch S"));
        RET(s->sat_scr.alloc((size_t)Np * 8, "scratch sat counts"));
        s->scr_Np = Np;
    }
    return TSAT_OK;
}

static int32_t reset_ctrl(tsat_solver* s, int64_t t)
{
    Ctrl c{};
    c.t = t;
    c.first_sat_step = -1;
    c.first_conv_step = -1;
    c.best_cand = 0;
    c.sat_cand = -1;
    HIPCHK(hipMemcpyAsync(s->ctrl.p, &c, sizeof c, hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

static int32_t binarize_current(tsat_solver* s, int32_t mode)
{
    tsat_params p = s->params;
    p.norm_mode = mode;
    VarArgs a = var_args(s, p, s->N, s->W, s->Np);
    a.lits_next = s->lits[s->cur].as<uint64_t>();
    a.theta = s->theta.as<float>();
    a.ctrl = s->ctrl.as<Ctrl>();
    HIPCHK(launch_var(a, VOP_BINARIZE, var_blocks(s, s->st.V), s->stream));
    s->bits_mode = mode;
    return TSAT_OK;
}

// the bits of the batch follow the normalization mode of the call using them
static int32_t ensure_mode(tsat_solver* s, int32_t mode)
{
    if (s->bits_mode == mode) return TSAT_OK;
    return binarize_current(s, mode);
}

// ---------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* tsat_last_error(void) { return g_err.c_str(); }

int32_t tsat_version(void) { return 10000; }

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
    return TSAT_OK;
}

int32_t tsat_cnf_info_of(int32_t num_vars, int64_t num_lits, const int32_t* lits, tsat_cnf_info* out)
{
    g_err.clear();
    if (!out) return fail(TSAT_E_ARG, "out is NULL");
    Store st;
    RET(build_store(num_vars, num_lits, lits, st, false));
    tsat_cnf_info info{};
    info.num_vars = st.V;
    info.max_width = st.K;
    info.num_clauses = st.C;
    info.num_lits = st.L;
    info.num_empty = st.n_empty;
    info.num_dup_removed = st.n_dup;
    info.num_tautologies = st.n_taut;
    for (int k = 0; k <= TSAT_MAX_WIDTH; ++k) info.width_count[k] = st.width_count[k];
    *out = info;
    return TSAT_OK;
}

int32_t tsat_dimacs_read(const char* path, int32_t* num_vars, int64_t* num_lits, int32_t* lits, int64_t cap)
{
    g_err.clear();
    if (!path || !num_vars || !num_lits) return fail(TSAT_E_ARG, "NULL argument");
    FILE* f = fopen(path, "rb");
    if (!f) return fail(TSAT_E_ARG, "cannot open %s", path);
    std::string text;
    char buf[1 << 16];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    long long hv = -1, hc = -1;
    int64_t count = 0, clauses = 0;
    bool open_clause = false;
    size_t pos = 0, line = 0;
    const size_t n = text.size();
    while (pos < n) {
        size_t eol = text.find('\n', pos);
        if (eol == std::string::npos) eol = n;
        ++line;
        size_t a = pos;
        while (a < eol && (text[a] == ' ' || text[a] == '\t' || text[a] == '\r')) ++a;
        if (a < eol && text[a] == 'c') { pos = eol + 1; continue; }
        if (a < eol && text[a] == '%') break; // end-of-data marker of some collections
        if (a < eol && text[a] == 'p') {
            if (hv >= 0) return fail(TSAT_E_PARSE, "line %zu: second header", line);
            char fmt[16] = {0};
            if (sscanf(text.c_str() + a, "p %15s %lld %lld", fmt, &hv, &hc) != 3 || strcmp(fmt, "cnf") != 0 || hv < 1 ||
                hv > 0x3fffffff || hc < 0)
                return fail(TSAT_E_PARSE, "line %zu: malformed header", line);
            pos = eol + 1;
            continue;
        }
        while (a < eol) {
            while (a < eol && (text[a] == ' ' || text[a] == '\t' || text[a] == '\r')) ++a;
            if (a >= eol) break;
            if (hv < 0) return fail(TSAT_E_PARSE, "line %zu: clause before the 'p cnf' header", line);
            char* end = nullptr;
            const long long x = strtoll(text.c_str() + a, &end, 10);
            const size_t used = (size_t)(end - (text.c_str() + a));
            if (used == 0 || (a + used < eol && !(text[a + used] == ' ' || text[a + used] == '\t' || text[a + used] == '\r')))
                return fail(TSAT_E_PARSE, "line %zu: invalid token", line);
            a += used;
            if (x > hv || x < -hv) return fail(TSAT_E_PARSE, "line %zu: literal %lld out of range", line, x);
            if (lits) {
                if (count >= cap) return fail(TSAT_E_ARG, "capacity %lld too small", (long long)cap);
                lits[count] = (int32_t)x;
            }
            ++count;
            if (x == 0) { ++clauses; open_clause = false; }
            else open_clause = true;
        }
        pos = eol + 1;
    }
    if (hv < 0) return fail(TSAT_E_PARSE, "missing 'p cnf' header");
    if (open_clause) {
        // a final clause without its 0 terminator is accepted and closed
        if (lits) {
            if (count >= cap) return fail(TSAT_E_ARG, "capacity %lld too small", (long long)cap);
            lits[count] = 0;
        }
        ++count;
        ++clauses;
    }
    if (clauses != hc) return fail(TSAT_E_PARSE, "header declares %lld clauses, found %lld", hc, (long long)clauses);
    *num_vars = (int32_t)hv;
    *num_lits = count;
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

int32_t tsat_load_cnf(tsat_solver* s, int32_t num_vars, int64_t num_lits, const int32_t* lits)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    RET(set_dev(s));
    Store st;
    RET(build_store(num_vars, num_lits, lits, st, true));
    HIPCHK(hipStreamSynchronize(s->stream));
    // drop the previous instance and batch
    for (auto* b : s->buckets) delete b;
    s->buckets.clear();
    s->loaded = false;
    s->N = s->W = s->Np = 0;
    s->scr_Np = 0;
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
    RET(s->occ_off.alloc(((size_t)s->st.V + 1) * 4, "occurrence offsets"));
    RET(s->occ_mid.alloc((size_t)s->st.V * 4, "occurrence offsets"));
    HIPCHK(hipMemcpy(s->occ_off.p, s->st.occ_off.data(), ((size_t)s->st.V + 1) * 4, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->occ_mid.p, s->st.occ_mid.data(), (size_t)s->st.V * 4, hipMemcpyHostToDevice));
    RET(s->occ_data.alloc(std::max<size_t>(4, s->st.occ_data.size() * 4), "occurrence records"));
    if (!s->st.occ_data.empty())
        HIPCHK(hipMemcpy(s->occ_data.p, s->st.occ_data.data(), s->st.occ_data.size() * 4, hipMemcpyHostToDevice));
    RET(s->witness.alloc((size_t)s->st.V, "witness"));
    s->loaded = true;
    return TSAT_OK;
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
    const size_t VN = (size_t)s->st.V * N;
    if ((size_t)K1 * Np * 4 > 64 * 1024)
        return fail(TSAT_E_ARG, "(max_width+1) * 64*ceil(N/64) * 4 bytes = %zu exceeds the 64 KiB table limit",
                    (size_t)K1 * Np * 4);
    RET(check_row_offsets(s, W));
    RET(s->lits[0].alloc((size_t)2 * s->st.V * W * 8, "literal rows"));
    RET(s->lits[1].alloc((size_t)2 * s->st.V * W * 8, "literal rows"));
    RET(s->theta.alloc(VN * 4, "theta"));
    RET(s->m.alloc(VN * 4, "m"));
    RET(s->v.alloc(VN * 4, "v"));
    RET(s->H.alloc((size_t)Np * K1 * 4, "histogram"));
    RET(s->H_last.alloc((size_t)Np * K1 * 4, "histogram"));
    RET(s->table.alloc((size_t)Np * K1 * 4, "table"));
    RET(s->S64.alloc((size_t)Np * 8, "S"));
    RET(s->sat.alloc((size_t)Np * 8, "sat counts"));
    HIPCHK(launch_fill_u32(s->H.as<uint32_t>(), (int64_t)Np * K1, 0u, s->stream));
    HIPCHK(launch_fill_u32(s->H_last.as<uint32_t>(), (int64_t)Np * K1, 0u, s->stream));
    HIPCHK(launch_fill_u32(s->m.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
    HIPCHK(launch_fill_u32(s->v.as<uint32_t>(), (int64_t)VN, 0u, s->stream));
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
    const size_t VN = (size_t)s->st.V * N;
    if (init_logits) HIPCHK(hipMemcpyAsync(s->theta.p, init_logits, VN * 4, hipMemcpyHostToDevice, s->stream));
    else HIPCHK(launch_init_normal(s->theta.as<float>(), (int64_t)VN, seed, s->stream));
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
    host.stop_on_sat = stop_on_sat ? 1 : 0;
    HIPCHK(hipMemcpyAsync(ctrl, &host, sizeof host, hipMemcpyHostToDevice, s->stream));

    SminArgs sa = smin_args(s, p, s->N, s->Np);
    sa.H = s->H.as<uint32_t>();
    sa.H_last = s->H_last.as<uint32_t>();
    sa.table = s->table.as<float>();
    sa.S64_out = s->S64.as<double>();
    sa.sat_out = s->sat.as<int64_t>();
    sa.ctrl = ctrl;
    sa.update = 1;
    VarArgs va = var_args(s, p, s->N, s->W, s->Np);
    va.tbl = s->table.as<float>();
    va.theta = s->theta.as<float>();
    va.m = s->m.as<float>();
    va.v = s->v.as<float>();
    va.ctrl = ctrl;
    va.witness = s->witness.as<uint8_t>();
    const int vblocks = var_blocks(s, s->st.V);

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
    for (int32_t it = 0; it < max_steps; ++it) {
        ++executed;
        RET(enqueue_fwd(s, s->lits[s->cur].as<uint64_t>(), s->W, s->H.as<uint32_t>(), ctrl, s->stream));
        if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 1], s->stream));
        HIPCHK(launch_smin(sa, s->stream));
        if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 2], s->stream));
        va.lits_cur = s->lits[s->cur].as<uint64_t>();
        va.lits_next = s->lits[1 - s->cur].as<uint64_t>();
        HIPCHK(launch_var(va, VOP_STEP, vblocks, s->stream));
        if (timing) HIPCHK(hipEventRecord(s->events[3 * it + 3], s->stream));
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
        tsat_report r{};
        r.steps_done = host.updates - updates0;
        r.first_sat_step = host.first_sat_step;
        r.first_converged_step = host.first_conv_step;
        r.best_sat_count = host.best_sat;
        r.next_step = host.t;
        r.loss = host.loss;
        r.best_candidate = host.best_cand;
        r.sat_candidate = host.sat_cand;
        r.nonfinite = host.nonfinite;
        *report = r;
    }
    if (host.nonfinite) return fail(TSAT_E_NUMERIC, "a logit or optimizer moment became non-finite");
    return TSAT_OK;
}

// stateless forward + SmoothMin of literal rows `lits` (N candidates)
static int32_t eval_rows(tsat_solver* s, const tsat_params& p, const uint64_t* lits, int32_t N, const float* dS,
                         uint32_t* H_out, float* S32, double* S64, int64_t* sat, float* table, hipStream_t st)
{
    const int32_t W = (N + 63) / 64, Np = 64 * W;
    RET(enqueue_fwd(s, lits, W, s->H_scr.as<uint32_t>(), nullptr, st));
    SminArgs a = smin_args(s, p, N, Np);
    a.H = s->H_scr.as<uint32_t>();
    a.H_last = H_out;
    a.table = table;
    a.S_out = S32;
    a.S64_out = S64;
    a.sat_out = sat;
    a.dS = dS;
    a.ctrl = s->ctrl_scr.as<Ctrl>();
    a.update = 0;
    HIPCHK(launch_smin(a, st));
    return TSAT_OK;
}

int32_t tsat_check(tsat_solver* s, int64_t* sat_counts, uint8_t* is_sat)
{
    g_err.clear();
    RET(need_batch(s));
    RET(ensure_scratch(s, s->N));
    RET(eval_rows(s, s->params, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, nullptr, nullptr, nullptr,
                  s->sat_scr.as<int64_t>(), nullptr, s->stream));
    std::vector<int64_t> sat(s->N);
    HIPCHK(hipMemcpyAsync(sat.data(), s->sat_scr.p, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int32_t i = 0; i < s->N; ++i) {
        if (sat_counts) sat_counts[i] = sat[i];
        if (is_sat) is_sat[i] = sat[i] == s->st.C ? 1 : 0;
    }
    return TSAT_OK;
}

int32_t tsat_check_bits(tsat_solver* s, const uint64_t* packed, int32_t N, int64_t* sat_counts, uint8_t* is_sat)
{
    g_err.clear();
    if (!s) return fail(TSAT_E_ARG, "solver is NULL");
    if (!s->loaded) return fail(TSAT_E_STATE, "no CNF loaded");
    if (N < 1 || !packed) return fail(TSAT_E_ARG, "N must be >= 1 and packed non-NULL");
    RET(set_dev(s));
    const int32_t W = (N + 63) / 64;
    if ((size_t)K1_of(s) * 64 * W * 4 > (size_t)1 << 34) return fail(TSAT_E_ARG, "N too large");
    RET(ensure_scratch(s, N));
    const size_t vb = (size_t)s->st.V * W * 8;
    RET(s->tmp.reserve(vb, "packed input"));
    HIPCHK(hipMemcpyAsync(s->tmp.p, packed, vb, hipMemcpyHostToDevice, s->stream));
    HIPCHK(launch_expand(s->tmp.as<uint64_t>(), s->st.V, W, N, s->lits_scr.as<uint64_t>(), s->stream));
    RET(eval_rows(s, s->params, s->lits_scr.as<uint64_t>(), N, nullptr, nullptr, nullptr, nullptr, s->sat_scr.as<int64_t>(),
                  nullptr, s->stream));
    std::vector<int64_t> sat;
    try {
        sat.resize(N);
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed");
    }
    HIPCHK(hipMemcpyAsync(sat.data(), s->sat_scr.p, (size_t)N * 8, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int32_t i = 0; i < N; ++i) {
        if (sat_counts) sat_counts[i] = sat[i];
        if (is_sat) is_sat[i] = sat[i] == s->st.C ? 1 : 0;
    }
    return TSAT_OK;
}

int32_t tsat_get_bits(tsat_solver* s, uint64_t* packed)
{
    g_err.clear();
    RET(need_batch(s));
    if (!packed) return fail(TSAT_E_ARG, "packed is NULL");
    // even literal rows hold the variable values
    HIPCHK(hipMemcpy2DAsync(packed, (size_t)s->W * 8, s->lits[s->cur].p, (size_t)2 * s->W * 8, (size_t)s->W * 8, s->st.V,
                            hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return TSAT_OK;
}

int32_t tsat_get_assignment(tsat_solver* s, int32_t cand, uint8_t* vals)
{
    g_err.clear();
    RET(need_batch(s));
    if (cand < 0 || cand >= s->N || !vals) return fail(TSAT_E_ARG, "candidate %d outside [0, %d) or NULL output", cand, s->N);
    std::vector<uint64_t> col(s->st.V);
    HIPCHK(hipMemcpy2DAsync(col.data(), 8, s->lits[s->cur].as<uint64_t>() + (cand >> 6), (size_t)2 * s->W * 8, 8, s->st.V,
                            hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int32_t v = 0; v < s->st.V; ++v) vals[v] = (uint8_t)((col[v] >> (cand & 63)) & 1u);
    return TSAT_OK;
}

int32_t tsat_get_witness(tsat_solver* s, uint8_t* vals, int32_t* cand)
{
    g_err.clear();
    RET(need_batch(s));
    Ctrl host{};
    HIPCHK(hipMemcpyAsync(&host, s->ctrl.p, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (host.sat_cand < 0) return fail(TSAT_E_STATE, "no satisfying assignment found yet");
    if (cand) *cand = host.sat_cand;
    if (!vals) return TSAT_OK;
    if (host.stop) return tsat_get_assignment(s, host.sat_cand, vals);
    HIPCHK(hipMemcpy(vals, s->witness.p, (size_t)s->st.V, hipMemcpyDeviceToHost));
    return TSAT_OK;
}

int32_t tsat_num_candidates(const tsat_solver* s) { return s ? s->N : 0; }

int32_t tsat_max_width(const tsat_solver* s) { return (s && s->loaded) ? s->st.K : 0; }

int32_t tsat_set_logits(tsat_solver* s, const float* theta)
{
    g_err.clear();
    RET(need_batch(s));
    if (!theta) return fail(TSAT_E_ARG, "theta is NULL");
    HIPCHK(hipMemcpyAsync(s->theta.p, theta, (size_t)s->st.V * s->N * 4, hipMemcpyHostToDevice, s->stream));
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
    const size_t VN = (size_t)s->st.V * s->N;
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
    const size_t VN = (size_t)s->st.V * s->N;
    if (theta) HIPCHK(hipMemcpyAsync(theta, s->theta.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    if (m) HIPCHK(hipMemcpyAsync(m, s->m.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    if (v) HIPCHK(hipMemcpyAsync(v, s->v.p, VN * 4, hipMemcpyDeviceToHost, s->stream));
    Ctrl host{};
    HIPCHK(hipMemcpyAsync(&host, s->ctrl.p, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (t) *t = host.t;
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
    RET(s->tmp.reserve((size_t)s->Np * K1 * 4, "histogram copy"));
    RET(eval_rows(s, p, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, s->tmp.as<uint32_t>(), nullptr,
                  s->S64_scr.as<double>(), nullptr, nullptr, s->stream));
    std::vector<double> S64(s->N);
    HIPCHK(hipMemcpyAsync(S64.data(), s->S64_scr.p, (size_t)s->N * 8, hipMemcpyDeviceToHost, s->stream));
    if (hist) HIPCHK(hipMemcpyAsync(hist, s->tmp.p, (size_t)s->N * K1 * 4, hipMemcpyDeviceToHost, s->stream));
    Ctrl host{};
    HIPCHK(hipMemcpyAsync(&host, s->ctrl_scr.p, sizeof host, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    if (S) memcpy(S, S64.data(), (size_t)s->N * 8);
    if (loss) *loss = host.loss;
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
    const size_t VN = (size_t)s->st.V * s->N;
    RET(s->tmp.reserve(VN * 8, "gradient copies"));
    RET(eval_rows(s, p, s->lits[s->cur].as<uint64_t>(), s->N, nullptr, nullptr, nullptr, nullptr, nullptr,
                  s->table_scr.as<float>(), s->stream));
    VarArgs va = var_args(s, p, s->N, s->W, s->Np);
    va.tbl = s->table_scr.as<float>();
    va.theta = s->theta.as<float>();
    va.lits_cur = s->lits[s->cur].as<uint64_t>();
    va.U_out = s->tmp.as<float>();
    va.g_out = s->tmp.as<float>() + VN;
    va.g_transposed = 0;
    HIPCHK(launch_var(va, VOP_GRAD, var_blocks(s, s->st.V), s->stream));
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
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
    HIPCHK(launch_pack(assign, s->st.V, N, (N + 63) / 64, bits, 0, st));
    return TSAT_OK;
}

static int32_t dev_prepare(tsat_solver* s, const uint64_t* bits, int32_t N, hipStream_t st)
{
    RET(ensure_scratch(s, N));
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
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
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
    hipStream_t st = stream ? (hipStream_t)stream : s->stream;
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

// ------------------------------------------------------------------ timing

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

} // extern "C"
