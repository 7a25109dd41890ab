// Host-only checks of the clause/occurrence store builder and the DIMACS
// reader, built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_store_sanitized.py (no GPU, no HIP).  Every store is checked
// against a naive restatement: the sorted distinct literal codes of each
// clause, the width buckets, and per variable and sign the records of the
// clauses that hold the literal.  Prints "ALL OK" and exits 0 on success.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "tsat.h"
#include "tsat_err.h"
#include "tsat_store.h"

using namespace tsat_host;

static int g_fail = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        if (!(c)) {                                                               \
            std::fprintf(stderr, "%s:%d: CHECK failed: %s\n", __FILE__, __LINE__, #c); \
            ++g_fail;                                                             \
        }                                                                         \
    } while (0)

// xorshift64* stream for the random CNFs of this test
struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed * 0x9E3779B97F4A7C15ull + 1) {}
    uint64_t next()
    {
        s ^= s >> 12;
        s ^= s << 25;
        s ^= s >> 27;
        return s * 2685821657736338717ull;
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }
};

struct Inst {
    int32_t V;
    std::vector<std::vector<int32_t>> clauses;
};

static uint32_t code_of(int32_t x, uint32_t base)
{
    return x > 0 ? 2u * (base + (uint32_t)(x - 1)) : 2u * (base + (uint32_t)(-x - 1)) + 1u;
}

// Random instance: widths drawn from `widths`, literals with repeats and
// occasional tautologies when allowed.
static Inst random_inst(Rng& r, int32_t V, int C, const std::vector<int>& widths, bool messy)
{
    Inst in;
    in.V = V;
    for (int c = 0; c < C; ++c) {
        const int k = widths[(size_t)r.below((int)widths.size())];
        std::vector<int32_t> cl;
        for (int e = 0; e < k; ++e) {
            int32_t x = 1 + r.below(V);
            if (r.below(2)) x = -x;
            cl.push_back(x);
        }
        if (messy && k > 0 && r.below(8) == 0) cl.push_back(cl[0]);   // repeated literal
        if (messy && k > 0 && r.below(16) == 0) cl.push_back(-cl[0]); // tautology
        in.clauses.push_back(cl);
    }
    return in;
}

static void stream_of(const std::vector<Inst>& insts, std::vector<int32_t>& nv, std::vector<int64_t>& off,
                      std::vector<int32_t>& lits)
{
    nv.clear();
    off.assign(1, 0);
    lits.clear();
    for (const auto& in : insts) {
        nv.push_back(in.V);
        for (const auto& cl : in.clauses) {
            lits.insert(lits.end(), cl.begin(), cl.end());
            lits.push_back(0);
        }
        off.push_back((int64_t)lits.size());
    }
}

// Compare a store with the naive restatement of the instances.
static void check_store(const std::vector<Inst>& insts, const Store& st, bool expect_occ)
{
    // expected clauses per width, per instance, as sorted distinct codes
    std::vector<std::vector<std::multiset<std::vector<uint32_t>>>> want(TSAT_MAX_WIDTH + 1);
    for (auto& w : want) w.resize(insts.size());
    int64_t C = 0, L = 0, n_dup = 0, n_taut = 0, n_empty = 0;
    int K = 0;
    uint32_t base = 0;
    for (size_t j = 0; j < insts.size(); ++j) {
        for (const auto& cl : insts[j].clauses) {
            std::vector<uint32_t> c;
            for (int32_t x : cl) c.push_back(code_of(x, base));
            std::sort(c.begin(), c.end());
            const size_t before = c.size();
            c.erase(std::unique(c.begin(), c.end()), c.end());
            n_dup += (int64_t)(before - c.size());
            bool taut = false;
            for (size_t e = 1; e < c.size(); ++e) taut |= (c[e] >> 1) == (c[e - 1] >> 1);
            n_taut += taut;
            n_empty += c.empty();
            K = std::max(K, (int)c.size());
            L += (int64_t)c.size();
            ++C;
            want[c.size()][j].insert(c);
        }
        CHECK(st.var_base[j] == base);
        base += (uint32_t)insts[j].V;
    }
    CHECK(st.V == (int32_t)base);
    CHECK(st.C == C);
    CHECK(st.L == L);
    CHECK(st.K == K);
    CHECK(st.n_dup == n_dup);
    CHECK(st.n_taut == n_taut);
    CHECK(st.n_empty == n_empty);
    // buckets: per instance range, the same multiset of clauses, in
    // lexicographic order
    for (int k = 0; k <= TSAT_MAX_WIDTH; ++k) {
        int64_t cnt = 0;
        for (size_t j = 0; j < insts.size(); ++j) {
            const int64_t c0 = st.inst_off[k][j], c1 = st.inst_off[k][j + 1];
            CHECK(c1 - c0 == (int64_t)want[k][j].size());
            cnt += c1 - c0;
            if (k == 0) continue;
            std::multiset<std::vector<uint32_t>> got;
            std::vector<uint32_t> prev;
            for (int64_t c = c0; c < c1; ++c) {
                std::vector<uint32_t> cl(st.buckets[k].begin() + c * k, st.buckets[k].begin() + (c + 1) * k);
                if (c > c0 && k >= 2) CHECK(!(cl < prev)); // widths >= 2 are ordered
                prev = cl;
                got.insert(cl);
            }
            CHECK(got == want[k][j]);
        }
        CHECK(st.width_count[k] == cnt);
    }
    if (!expect_occ) return;
    // occurrence records: per variable and sign, one record per clause
    // holding the literal, naming the clause's other literals
    std::map<uint32_t, std::multiset<std::vector<uint32_t>>> occ_want, occ_got;
    for (int k = 1; k <= st.K; ++k) {
        const size_t Cb = st.buckets[k].size() / (size_t)k;
        for (size_t c = 0; c < Cb; ++c) {
            const uint32_t* cl = &st.buckets[k][c * k];
            for (int e = 0; e < k; ++e) {
                std::vector<uint32_t> rest;
                for (int f = 0; f < k; ++f)
                    if (f != e) rest.push_back(cl[f]);
                occ_want[cl[e]].insert(rest);
            }
        }
    }
    const bool pure = st.pure_k != 0;
    for (int32_t v = 0; v < st.V; ++v) {
        const uint32_t b = st.occ_off[v], m = st.occ_mid[v], e = st.occ_off[v + 1];
        CHECK(b <= m && m <= e);
        for (int sg = 0; sg < 2; ++sg) {
            const uint32_t lit = 2u * (uint32_t)v + (uint32_t)sg;
            uint32_t q = sg ? m : b;
            const uint32_t end = sg ? e : m;
            while (q < end) {
                std::vector<uint32_t> rest;
                if (pure) {
                    const size_t w = (size_t)q * (size_t)(st.pure_k - 1);
                    rest.assign(st.occ_data.begin() + (ptrdiff_t)w, st.occ_data.begin() + (ptrdiff_t)(w + st.pure_k - 1));
                    q += 1;
                } else {
                    const uint32_t k1 = st.occ_data[q];
                    rest.assign(st.occ_data.begin() + q + 1, st.occ_data.begin() + q + 1 + k1);
                    q += 1 + k1;
                }
                occ_got[lit].insert(rest);
            }
            CHECK(q == end);
        }
    }
    CHECK(occ_got == occ_want);
    // clause-index records: per variable and sign, exactly the global
    // indices of the clauses holding the literal
    if (st.K >= 1 && st.K <= kMaxPlaneWidth) {
        CHECK(!st.plane_base.empty());
        std::map<uint32_t, std::multiset<int64_t>> cid_want, cid_got;
        int64_t base = 0;
        for (int k = 1; k <= TSAT_MAX_WIDTH; ++k) {
            CHECK(st.plane_base[k] == base);
            if (k <= st.K) {
                const size_t Cb = st.buckets[k].size() / (size_t)k;
                for (size_t c = 0; c < Cb; ++c)
                    for (int e = 0; e < k; ++e) cid_want[st.buckets[k][c * k + e]].insert(base + (int64_t)c);
            }
            base += st.width_count[k];
        }
        CHECK(st.plane_clauses == base);
        const std::vector<uint32_t>& off = pure ? st.occ_off : st.cid_off;
        const std::vector<uint32_t>& mid = pure ? st.occ_mid : st.cid_mid;
        CHECK(off.size() == (size_t)st.V + 1 && off[st.V] == st.occ_cid.size());
        uint64_t most = 0;
        for (int32_t v = 0; v < st.V; ++v) {
            CHECK(off[v] <= mid[v] && mid[v] <= off[v + 1]);
            most = std::max<uint64_t>(most, std::max(mid[v] - off[v], off[v + 1] - mid[v]));
            for (uint32_t q = off[v]; q < off[v + 1]; ++q) {
                CHECK((int64_t)st.occ_cid[q] < st.plane_clauses);
                cid_got[2u * (uint32_t)v + (q >= mid[v] ? 1u : 0u)].insert(st.occ_cid[q]);
            }
        }
        CHECK(most == st.max_sign_rec);
        CHECK(cid_got == cid_want);
    } else {
        CHECK(st.occ_cid.empty());
    }
    // heavy chunks of generic stores tile each heavy variable's records
    if (!pure && !st.hv_var.empty()) {
        for (size_t h = 0; h < st.hv_var.size(); ++h) {
            const uint32_t v = st.hv_var[h];
            CHECK(st.heavy[v] == 1u);
            uint32_t q = st.occ_off[v];
            for (uint32_t c = st.hv_chunk[h]; c < st.hv_chunk[h + 1]; ++c) {
                CHECK(st.ch_var[c] == v);
                CHECK(st.ch_beg[c] == q);
                q = st.ch_end[c];
            }
            CHECK(q == st.occ_off[v + 1]);
        }
    }
}

static void test_random_stores()
{
    Rng r(7);
    const std::vector<std::vector<int>> width_sets = {{3}, {2}, {4}, {1, 2, 3}, {0, 2, 5, 12}, {1, 32}, {2, 3, 7}};
    for (int trial = 0; trial < 40; ++trial) {
        const auto& ws = width_sets[(size_t)trial % width_sets.size()];
        const int n_inst = 1 + r.below(4);
        std::vector<Inst> insts;
        for (int j = 0; j < n_inst; ++j) {
            const int32_t V = 1 + r.below(60);
            const bool wide = std::find(ws.begin(), ws.end(), 32) != ws.end();
            const int32_t Vw = wide ? std::max(V, 40) : V;
            insts.push_back(random_inst(r, Vw, r.below(300), ws, trial % 2 == 1));
        }
        // keep widths distinct-safe: clauses wider than V collapse by de-duplication
        std::vector<int32_t> nv, lits;
        std::vector<int64_t> off;
        stream_of(insts, nv, off, lits);
        Store st;
        const int32_t rc = build_store(n_inst, nv.data(), off.data(), lits.data(), st, true);
        CHECK(rc == TSAT_OK);
        if (rc == TSAT_OK) check_store(insts, st, true);
    }
}

// A variable in many clauses: generic stores cut it into chunks.
static void test_heavy_variable()
{
    Inst in;
    in.V = 50;
    Rng r(11);
    for (int c = 0; c < 900; ++c) in.clauses.push_back({1, 2 + r.below(49), -(2 + r.below(49)), 2 + r.below(49), 5});
    std::vector<int32_t> nv, lits;
    std::vector<int64_t> off;
    stream_of({in}, nv, off, lits);
    Store st;
    CHECK(build_store(1, nv.data(), off.data(), lits.data(), st, true) == TSAT_OK);
    CHECK(!st.hv_var.empty());
    check_store({in}, st, true);
}

// Header-less records past the byte limit become generic records; a store
// past the word limit is refused.
static void test_limits()
{
    Rng r(3);
    Inst in;
    in.V = 40;
    for (int c = 0; c < 200; ++c) {
        const int32_t a = 1 + r.below(38); // three distinct variables
        in.clauses.push_back({a, -(a + 1), r.below(2) ? a + 2 : -(a + 2)});
    }
    std::vector<int32_t> nv, lits;
    std::vector<int64_t> off;
    stream_of({in}, nv, off, lits);
    Store st;
    CHECK(build_store(1, nv.data(), off.data(), lits.data(), st, true) == TSAT_OK);
    CHECK(st.pure_k == 3 && !st.occ_cid.empty());
    StoreLimits lim;
    lim.max_pure_bytes = (uint64_t)st.L * 2 * 4 - 1; // one byte short of the header-less records
    Store g;
    CHECK(build_store(1, nv.data(), off.data(), lits.data(), g, true, lim) == TSAT_OK);
    CHECK(g.pure_k == 0 && g.occ_cid.size() == (size_t)g.L && g.cid_off.size() == (size_t)g.V + 1);
    CHECK(g.occ_data.size() == (size_t)g.L * 3);
    check_store({in}, g, true);
    lim.max_pure_bytes = (uint64_t)st.L * 2 * 4; // exactly fits
    Store p;
    CHECK(build_store(1, nv.data(), off.data(), lits.data(), p, true, lim) == TSAT_OK);
    CHECK(p.pure_k == 3);
    StoreLimits tight;
    tight.max_occ_words = (uint64_t)st.L * 2 - 1;
    Store t;
    CHECK(build_store(1, nv.data(), off.data(), lits.data(), t, true, tight) == TSAT_E_ARG);
    CHECK(g_err.find("occurrence store exceeds") != std::string::npos);
}

static void test_errors()
{
    Store st;
    {
        const int32_t nv = 3;
        const int32_t lits[] = {1, -4, 0};
        const int64_t off[] = {0, 3};
        CHECK(build_store(1, &nv, off, lits, st, true) == TSAT_E_ARG); // |lit| > V
    }
    {
        const int32_t nv = 3;
        const int32_t lits[] = {1, 2};
        const int64_t off[] = {0, 2};
        CHECK(build_store(1, &nv, off, lits, st, true) == TSAT_E_ARG); // unterminated
    }
    {
        const int32_t nv = 0;
        const int64_t off[] = {0, 0};
        CHECK(build_store(1, &nv, off, nullptr, st, true) == TSAT_E_ARG); // no variables
    }
    {
        std::vector<int32_t> lits;
        for (int x = 1; x <= 33; ++x) lits.push_back(x);
        lits.push_back(0);
        const int32_t nv = 40;
        const int64_t off[] = {0, (int64_t)lits.size()};
        CHECK(build_store(1, &nv, off, lits.data(), st, true) == TSAT_E_ARG); // 33 distinct literals
        lits.insert(lits.begin(), 1); // a repeat does not count
        lits.erase(lits.begin() + 33);
        const int64_t off2[] = {0, (int64_t)lits.size()};
        CHECK(build_store(1, &nv, off2, lits.data(), st, true) == TSAT_OK);
        CHECK(st.K == 32 && st.n_dup == 1);
    }
    {
        // empty clauses and a CNF without clauses
        const int32_t nv = 2;
        const int32_t lits[] = {0, 1, -2, 0, 0};
        const int64_t off[] = {0, 5};
        CHECK(build_store(1, &nv, off, lits, st, true) == TSAT_OK);
        CHECK(st.n_empty == 2 && st.C == 3 && st.L == 2);
        const int64_t off0[] = {0, 0};
        CHECK(build_store(1, &nv, off0, nullptr, st, true) == TSAT_OK);
        CHECK(st.C == 0 && st.L == 0);
    }
}

static std::string write_tmp(const std::string& dir, const char* name, const char* text)
{
    const std::string path = dir + "/" + name;
    FILE* f = std::fopen(path.c_str(), "wb");
    if (!f) return path;
    std::fputs(text, f);
    std::fclose(f);
    return path;
}

static void test_dimacs(const std::string& dir)
{
    int32_t V = 0;
    int64_t n = 0;
    const std::string good = write_tmp(dir, "good.cnf", "c comment\np cnf 4 3\n1 -2 0\n3 4\n -1 0\n\t2 -4 0\n");
    CHECK(tsat_dimacs_read(good.c_str(), &V, &n, nullptr, 0) == TSAT_OK);
    CHECK(V == 4 && n == 10);
    std::vector<int32_t> buf((size_t)n);
    CHECK(tsat_dimacs_read(good.c_str(), &V, &n, buf.data(), n) == TSAT_OK);
    const std::vector<int32_t> want = {1, -2, 0, 3, 4, -1, 0, 2, -4, 0};
    CHECK(buf == want);
    CHECK(tsat_dimacs_read(good.c_str(), &V, &n, buf.data(), n - 1) == TSAT_E_ARG); // capacity
    // a final clause without its terminator is closed
    const std::string open_end = write_tmp(dir, "open.cnf", "p cnf 2 2\n1 2 0\n-1");
    CHECK(tsat_dimacs_read(open_end.c_str(), &V, &n, nullptr, 0) == TSAT_OK);
    CHECK(n == 5);
    const char* bad[] = {"1 2 0\n",                        // no header
                         "p cnf 2 1\np cnf 2 1\n1 0\n",     // second header
                         "p cnf 2 1\n1 x 0\n",              // bad token
                         "p cnf 2 1\n1 3 0\n",              // out of range
                         "p cnf 2 2\n1 0\n",                // clause count
                         "p dnf 2 1\n1 0\n",                // format
                         "p cnf -1 1\n1 0\n",               // negative V
                         "p cnf 2 1\n12abc 0\n"};           // junk after a number
    int i = 0;
    for (const char* t : bad) {
        char name[32];
        std::snprintf(name, sizeof name, "bad%d.cnf", i++);
        const std::string p = write_tmp(dir, name, t);
        CHECK(tsat_dimacs_read(p.c_str(), &V, &n, nullptr, 0) == TSAT_E_PARSE);
    }
    CHECK(tsat_dimacs_read((dir + "/missing.cnf").c_str(), &V, &n, nullptr, 0) == TSAT_E_ARG);
    CHECK(tsat_dimacs_read(nullptr, &V, &n, nullptr, 0) == TSAT_E_ARG);
    // cnf info of the good file
    tsat_cnf_info info;
    CHECK(tsat_cnf_info_of(4, 10, want.data(), &info) == TSAT_OK);
    CHECK(info.num_clauses == 3 && info.num_lits == 7 && info.max_width == 3 && info.width_count[2] == 2);
}

// work items of the window gathers: contiguous runs covering every
// variable, each within the variable and record limits or a single
// variable, none extendable by the next variable
static void test_window_chunks()
{
    Rng r(17);
    for (int t = 0; t < 200; ++t) {
        const size_t V = (size_t)r.below(300);
        std::vector<uint32_t> off(V + 1, 0);
        for (size_t v = 0; v < V; ++v) {
            const uint32_t k = r.below(8) == 0 ? 60 + r.below(100) : r.below(20); // some heavy variables
            off[v + 1] = off[v] + k;
        }
        const size_t mv = 1 + r.below(10);
        const uint32_t mr = 1 + r.below(90);
        const std::vector<uint32_t> ch = window_chunks(off, V, mv, mr);
        CHECK(!ch.empty() && ch.front() == 0 && ch.back() == (uint32_t)V);
        for (size_t i = 0; i + 1 < ch.size(); ++i) {
            const size_t b = ch[i], e = ch[i + 1];
            CHECK(b < e);
            const bool fits = e - b <= mv && off[e] - off[b] <= mr;
            CHECK(fits || e - b == 1);
            if (fits && e < V) CHECK(e - b == mv || off[e + 1] - off[b] > mr); // greedy: could not take v = e
        }
    }
    CHECK(window_chunks(std::vector<uint32_t>{0}, 0).size() == 1);
}

int main(int argc, char** argv)
{
    test_window_chunks();
    const std::string dir = argc > 1 ? argv[1] : ".";
    test_random_stores();
    test_heavy_variable();
    test_limits();
    test_errors();
    test_dimacs(dir);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("ALL OK\n");
    return 0;
}
