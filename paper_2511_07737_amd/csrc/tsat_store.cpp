// tsat_store.cpp -- clause store, occurrence store and DIMACS reader of the
// gradient-guided SAT library (TurboSAT, arXiv 2511.07737): the host-only
// part of the C-ABI.  Plain C++ (no HIP), so that it also builds into the
// sanitizer-instrumented host test.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "tsat.h"
#include "tsat_err.h"
#include "tsat_store.h"

namespace tsat_host {

static inline uint32_t lit_code(int32_t x, uint32_t base)
{
    return x > 0 ? 2u * (base + (uint32_t)(x - 1)) : 2u * (base + (uint32_t)(-x - 1)) + 1u;
}

int32_t build_store(int32_t n_inst, const int32_t* num_vars, const int64_t* lit_off, const int32_t* lits,
                    Store& st, bool with_occ, const StoreLimits& lim)
{
    if (n_inst < 1 || !num_vars || !lit_off) return fail(TSAT_E_ARG, "invalid instance list");
    st = Store();
    st.n_inst = n_inst;
    st.var_base.assign((size_t)n_inst + 1, 0);
    st.info.assign((size_t)n_inst, tsat::InstInfo{0, 0});
    int64_t total_v = 0;
    for (int32_t j = 0; j < n_inst; ++j) {
        if (num_vars[j] < 1) return fail(TSAT_E_ARG, "num_vars must be >= 1 (instance %d has %d)", j, num_vars[j]);
        const int64_t n = lit_off[j + 1] - lit_off[j];
        if (n < 0 || (n > 0 && !lits)) return fail(TSAT_E_ARG, "invalid literal stream of instance %d", j);
        if (n > 0 && lits[lit_off[j + 1] - 1] != 0)
            return fail(TSAT_E_ARG, "the last clause of instance %d is not terminated by 0", j);
        st.var_base[j] = (uint32_t)total_v;
        total_v += num_vars[j];
        if (2 * total_v > (int64_t)0x7fffffff) return fail(TSAT_E_ARG, "too many variables (%lld)", (long long)total_v);
    }
    st.var_base[n_inst] = (uint32_t)total_v;
    st.V = (int32_t)total_v;
    std::vector<uint32_t> cl;
    std::vector<std::vector<uint32_t>> buckets(TSAT_MAX_WIDTH + 1);
    std::vector<std::vector<int64_t>> inst_cnt(TSAT_MAX_WIDTH + 1, std::vector<int64_t>((size_t)n_inst, 0));
    try {
        for (int32_t j = 0; j < n_inst; ++j) {
            const uint32_t base = st.var_base[j];
            const int32_t Vj = num_vars[j];
            int64_t start = lit_off[j];
            for (int64_t q = lit_off[j]; q < lit_off[j + 1]; ++q) {
                const int32_t x = lits[q];
                if (x != 0) {
                    const int64_t a = x < 0 ? -(int64_t)x : (int64_t)x;
                    if (a > Vj)
                        return fail(TSAT_E_ARG, "literal %d at position %lld exceeds num_vars=%d", x,
                                    (long long)(q - lit_off[j]), Vj);
                    continue;
                }
                cl.clear();
                for (int64_t e = start; e < q; ++e) cl.push_back(lit_code(lits[e], base));
                start = q + 1;
                std::sort(cl.begin(), cl.end());
                const size_t before = cl.size();
                cl.erase(std::unique(cl.begin(), cl.end()), cl.end());
                st.n_dup += (int64_t)(before - cl.size());
                for (size_t e = 1; e < cl.size(); ++e)
                    if ((cl[e] >> 1) == (cl[e - 1] >> 1)) { ++st.n_taut; break; }
                const size_t k = cl.size();
                if (k > TSAT_MAX_WIDTH)
                    return fail(TSAT_E_ARG, "clause %lld has %zu distinct literals (max %d)", (long long)st.C, k,
                                TSAT_MAX_WIDTH);
                buckets[k].insert(buckets[k].end(), cl.begin(), cl.end());
                st.width_count[k] += 1;
                inst_cnt[k][j] += 1;
                st.info[j].C += 1;
                if (k == 0) st.info[j].n_empty += 1;
                if ((int)k > st.K) st.K = (int)k;
                st.C += 1;
                st.L += (int64_t)k;
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed while building the clause store");
    }
    st.n_empty = st.width_count[0];
    st.buckets = std::move(buckets);
    st.inst_off.assign(TSAT_MAX_WIDTH + 1, std::vector<int64_t>((size_t)n_inst + 1, 0));
    for (int k = 0; k <= TSAT_MAX_WIDTH; ++k)
        for (int32_t j = 0; j < n_inst; ++j) st.inst_off[k][j + 1] = st.inst_off[k][j] + inst_cnt[k][j];
    // Within each instance and width, clauses in lexicographic order of their
    // (sorted) literal codes: a clause then sits next to the other clauses of
    // its smallest variable, so the forward's row gathers and the update's
    // plane gathers of neighbouring variables share cache lines.  The order
    // is internal: histograms and counts do not depend on it.
    try {
        std::vector<int64_t> idx;
        std::vector<uint32_t> tmp;
        for (int k = 2; k <= TSAT_MAX_WIDTH; ++k) {
            auto& b = st.buckets[k];
            for (int32_t j = 0; j < n_inst; ++j) {
                const int64_t c0 = st.inst_off[k][j], c1 = st.inst_off[k][j + 1];
                if (c1 - c0 < 2) continue;
                idx.resize((size_t)(c1 - c0));
                for (int64_t c = c0; c < c1; ++c) idx[(size_t)(c - c0)] = c;
                const uint32_t* base = b.data();
                std::sort(idx.begin(), idx.end(), [base, k](int64_t x, int64_t y) {
                    return std::lexicographical_compare(base + x * k, base + x * k + k, base + y * k, base + y * k + k);
                });
                tmp.resize((size_t)(c1 - c0) * k);
                for (size_t q = 0; q < idx.size(); ++q)
                    std::copy(base + idx[q] * k, base + idx[q] * k + k, tmp.begin() + (ptrdiff_t)(q * k));
                std::copy(tmp.begin(), tmp.end(), b.begin() + c0 * k);
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed while ordering the clause store");
    }
    if (!with_occ) return TSAT_OK;
    // per variable: records of positive occurrences, then negative ones;
    // record = (k-1, codes of the other k-1 literals), without the leading
    // k-1 when every clause has the same width
    {
        int64_t nonempty = 0;
        for (int k = 1; k <= TSAT_MAX_WIDTH; ++k) nonempty += st.width_count[k];
        if (st.K >= 2 && st.K <= 4 && st.width_count[st.K] == nonempty) st.pure_k = st.K;
        // header-less records are addressed by 32-bit byte offsets: past the
        // limit the store takes generic records
        if (st.pure_k && (uint64_t)st.L * (uint64_t)(st.pure_k - 1) * 4u > lim.max_pure_bytes) st.pure_k = 0;
    }
    const bool pure = st.pure_k != 0;
    const int32_t V = st.V;
    try {
        std::vector<uint64_t> wpos(V, 0), wneg(V, 0);
        for (int k = 1; k <= st.K; ++k) {
            const auto& b = st.buckets[k];
            for (size_t q = 0; q < b.size(); ++q) {
                const uint32_t c = b[q];
                (c & 1u ? wneg : wpos)[c >> 1] += pure ? 1u : (uint64_t)k;
            }
        }
        uint64_t total = 0;
        st.occ_off.assign((size_t)V + 1, 0);
        st.occ_mid.assign((size_t)V, 0);
        for (int32_t v = 0; v < V; ++v) {
            st.occ_off[v] = (uint32_t)total;
            st.occ_mid[v] = (uint32_t)(total + wpos[v]);
            st.max_sign_deg = std::max(st.max_sign_deg, std::max(wpos[v], wneg[v]));
            total += wpos[v] + wneg[v];
            if (total > lim.max_occ_words)
                return fail(TSAT_E_ARG, "occurrence store exceeds %llu words", (unsigned long long)lim.max_occ_words);
        }
        st.occ_off[V] = (uint32_t)total;
        // pure records are counted in records; the array holds (k-1) words each
        const uint64_t words = pure ? total * (uint64_t)(st.pure_k - 1) : total;
        if (words > lim.max_occ_words)
            return fail(TSAT_E_ARG, "occurrence store exceeds %llu words", (unsigned long long)lim.max_occ_words);
        st.occ_data.assign(words, 0);
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
                    if (pure) {
                        size_t w = (size_t)pos * (size_t)(k - 1);
                        for (int f = 0; f < k; ++f)
                            if (f != e) st.occ_data[w++] = lit[f];
                        ++pos;
                    } else {
                        st.occ_data[pos++] = (uint32_t)(k - 1);
                        for (int f = 0; f < k; ++f)
                            if (f != e) st.occ_data[pos++] = lit[f];
                    }
                }
            }
        }
        if (!pure) {
            st.heavy.assign((size_t)V, 0u);
            st.hv_chunk.push_back(0);
            for (int32_t v = 0; v < V; ++v) {
                const uint32_t b = st.occ_off[v], e = st.occ_off[v + 1];
                if (e - b <= kHeavyWords) continue;
                st.heavy[v] = 1u;
                st.hv_var.push_back((uint32_t)v);
                uint32_t q = b, cb = b;
                while (q < e) {
                    const uint32_t len = 1u + st.occ_data[q];
                    if (q > cb && q + len - cb > kChunkWords) {
                        st.ch_var.push_back((uint32_t)v);
                        st.ch_beg.push_back(cb);
                        st.ch_end.push_back(q);
                        cb = q;
                    }
                    q += len;
                }
                st.ch_var.push_back((uint32_t)v);
                st.ch_beg.push_back(cb);
                st.ch_end.push_back(e);
                st.hv_chunk.push_back((uint32_t)st.ch_var.size());
            }
            if (st.hv_var.empty()) {
                st.heavy.clear();
                st.hv_chunk.clear();
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(TSAT_E_OOM, "host allocation failed while building the occurrence store");
    }
    // clause-index records for the plane gathers
    if (st.K >= 1 && st.K <= kMaxPlaneWidth && (uint64_t)st.L < 0xffffffffull && (uint64_t)st.C < 0xffffffffull) {
        try {
            st.plane_base.assign(TSAT_MAX_WIDTH + 1, 0);
            int64_t base = 0;
            for (int k = 1; k <= TSAT_MAX_WIDTH; ++k) {
                st.plane_base[k] = base;
                base += st.width_count[k];
            }
            st.plane_clauses = base;
            std::vector<uint32_t> npos(V, 0), nneg(V, 0);
            for (int k = 1; k <= st.K; ++k)
                for (const uint32_t c : st.buckets[k]) ++((c & 1u) ? nneg : npos)[c >> 1];
            std::vector<uint32_t> curp(V), curn(V);
            if (!pure) {
                st.cid_off.assign((size_t)V + 1, 0);
                st.cid_mid.assign((size_t)V, 0);
            }
            uint64_t total = 0;
            for (int32_t v = 0; v < V; ++v) {
                curp[v] = (uint32_t)total;
                curn[v] = (uint32_t)(total + npos[v]);
                if (!pure) {
                    st.cid_off[v] = curp[v];
                    st.cid_mid[v] = curn[v];
                }
                st.max_sign_rec = std::max<uint64_t>(st.max_sign_rec, std::max(npos[v], nneg[v]));
                total += (uint64_t)npos[v] + nneg[v];
            }
            if (!pure) st.cid_off[V] = (uint32_t)total;
            st.occ_cid.assign(total, 0);
            for (int k = 1; k <= st.K; ++k) {
                const auto& b = st.buckets[k];
                const size_t Cb = b.size() / (size_t)k;
                for (size_t c = 0; c < Cb; ++c)
                    for (int e = 0; e < k; ++e) {
                        const uint32_t code = b[c * k + e];
                        uint32_t& pos = (code & 1u) ? curn[code >> 1] : curp[code >> 1];
                        st.occ_cid[pos++] = (uint32_t)(st.plane_base[k] + (int64_t)c);
                    }
            }
        } catch (const std::bad_alloc&) {
            return fail(TSAT_E_OOM, "host allocation failed while building the clause-index records");
        }
    }
    return TSAT_OK;
}

std::vector<uint32_t> window_chunks(const std::vector<uint32_t>& off, size_t V, size_t max_vars, uint32_t max_records)
{
    std::vector<uint32_t> ch;
    for (size_t v = 0; v < V;) {
        size_t e = v;
        while (e < V && e - v < max_vars && off[e + 1] - off[v] <= max_records) ++e;
        if (e == v) e = v + 1;
        ch.push_back((uint32_t)v);
        v = e;
    }
    ch.push_back((uint32_t)V);
    return ch;
}

} // namespace tsat_host

using namespace tsat_host;

extern "C" {

int32_t tsat_cnf_info_of(int32_t num_vars, int64_t num_lits, const int32_t* lits, tsat_cnf_info* out)
{
    g_err.clear();
    if (!out) return fail(TSAT_E_ARG, "out is NULL");
    if (num_lits < 0) return fail(TSAT_E_ARG, "invalid literal stream (n=%lld)", (long long)num_lits);
    Store st;
    const int64_t off[2] = {0, num_lits};
    RET(build_store(1, &num_vars, off, lits, st, false));
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

} // extern "C"
