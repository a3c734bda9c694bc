// CPU check of the solver's host-side planning (host_plan.hpp), built with
// AddressSanitizer and UndefinedBehaviorSanitizer by test_host_plan_cpu.py:
// random batches (uniform and not, packed, gapped and permuted offsets,
// planted invalid entries) through plan_batch, random host-resident pieces
// through copy_runs, and the chunk capacity of memory-limited solves.  Every
// check states a property of the result, not the planner's formulas.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <set>
#include <thread>

#include "host_plan.hpp"

using namespace blp;

static int failures = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            ++failures;                                   \
            std::fprintf(stderr, "FAILED %s: ", #cond);   \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            if (failures > 20) std::exit(1);              \
        }                                                 \
    } while (0)

static const VariantShape kShapes[] = {{8, 8}, {7, 11}, {8, 8}, {16, 16}, {32, 32}, {64, 64}, {112, 112, 1},
                                       {112, 112}, {128, 112}, {128, 128}, {160, 160}};

// Threads mode (built with ThreadSanitizer by the test): one planner per
// thread, as with one handle per thread.  Random batches are planned once on
// the main thread; then four threads plan all of them at once, each with its
// own reused Plan and in its own order, and every result must equal the
// serial one (the planner keeps no state outside its arguments).
struct Case {
    std::vector<int32_t> m, n, kind;
    std::vector<int64_t> ao, ro, co;
    PlanIn in;
};
static std::string digest(int rc, const Plan& p, bool uni) {
    if (rc != PLAN_OK) return std::to_string(rc) + "|" + p.msg;  // a refused batch: the code and message only
    char buf[256];
    std::snprintf(buf, sizeof buf, "%d|%d|%d|%lld|%lld|%lld|%lld|%d|%d|%lld|%lld|%d|%d|", rc, (int)p.any_simplex,
                  (int)p.any_box, (long long)p.n_box, (long long)p.tot_a, (long long)p.tot_m, (long long)p.tot_n,
                  p.max_m, p.max_cols, (long long)p.max_slot, (long long)p.n_may_stream, (int)p.gm_deep, p.box_n);
    std::string d = buf + p.msg + "|";
    if (uni) return d;  // a uniform batch's offsets are implied (the vectors are not used)
    for (size_t k = 0; k < p.a_off.size(); ++k)
        d += std::to_string(p.a_off[k]) + "," + std::to_string(p.row_off[k]) + "," + std::to_string(p.col_off[k]) + ";";
    return d;
}
static int threads_main() {
    std::mt19937_64 rng(7);
    auto U = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
    const int kNreg = (int)(sizeof kShapes / sizeof kShapes[0]);
    std::vector<Case> cases(400);
    for (Case& c : cases) {
        const int64_t K = U(0, 50);
        const bool uni = U(0, 3) == 0;
        c.m.resize(K), c.n.resize(K), c.kind.resize(K), c.ao.resize(K), c.ro.resize(K), c.co.resize(K);
        int64_t a = 0, r = 0, cc = 0;
        for (int64_t k = 0; k < K; ++k) {
            c.kind[k] = U(0, 4) == 0 ? 1 : 0;
            c.n[k] = uni && k ? c.n[0] : U(1, 300);
            c.m[k] = c.kind[k] ? 0 : (uni && k ? c.m[0] : U(1, 300));
            if (uni && k) c.kind[k] = c.kind[0], c.m[k] = c.m[0];
            if (U(0, 20) == 0) c.m[k] = 5000;  // an invalid entry now and then
            a += U(0, 3), r += U(0, 3), cc += U(0, 3);
            c.ao[k] = a, c.ro[k] = r, c.co[k] = cc;
            a += (int64_t)c.m[k] * c.n[k], r += c.m[k], cc += c.n[k];
        }
        c.in.count = K;
        c.in.uniform = uni;
        c.in.has_A = c.in.has_b = c.in.has_sense = c.in.has_c = c.in.has_l = c.in.has_u = true;
        c.in.variants = kShapes;
        c.in.nreg = kNreg;
        c.in.force = U(0, 5) == 0 ? U(-2, kNreg - 1) : -1;
        c.in.lpc = U(0, 3) != 0;
    }
    for (Case& c : cases) {  // pointers once the vectors are final
        c.in.m = c.m.data(), c.in.n = c.n.data(), c.in.kind = c.kind.data();
        if (!c.in.uniform && c.m.size() % 2) c.in.a_off = c.ao.data(), c.in.row_off = c.ro.data(), c.in.col_off = c.co.data();
    }
    std::vector<std::string> want(cases.size());
    {
        Plan p;
        for (size_t i = 0; i < cases.size(); ++i) want[i] = digest(plan_batch(cases[i].in, p), p, cases[i].in.uniform);
    }
    constexpr int kThreads = 4;
    std::vector<int> bad(kThreads, 0);
    std::vector<std::thread> th;
    for (int t = 0; t < kThreads; ++t)
        th.emplace_back([&, t] {
            Plan p;
            std::vector<int64_t> order;
            std::vector<CopyRun> runs;
            for (int rep = 0; rep < 3; ++rep)
                for (size_t q = 0; q < cases.size(); ++q) {
                    const size_t i = (q * (2 * t + 1) + (size_t)rep * 97) % cases.size();
                    if (digest(plan_batch(cases[i].in, p), p, cases[i].in.uniform) != want[i]) ++bad[t];
                    if (!cases[i].in.uniform && p.code == PLAN_OK && !p.a_off.empty()) {
                        std::vector<int32_t> len(cases[i].n.begin(), cases[i].n.end());
                        int64_t lo = INT64_MAX;
                        for (int64_t o : p.col_off) lo = std::min(lo, o);
                        copy_runs(p.col_off, len, 0, (int64_t)len.size(), lo, order, runs);
                        int64_t tot = 0;
                        for (const CopyRun& r : runs) tot += r.len;
                        int64_t sum = 0;
                        for (int32_t l : len) sum += l;
                        if (tot != sum) ++bad[t];
                    }
                }
        });
    for (std::thread& x : th) x.join();
    int total = 0;
    for (int b : bad) total += b;
    std::printf("host plan threads: %d failures\n", total);
    return total ? 1 : 0;
}

int main(int argc, char** argv) {
    if (argc > 1 && std::strcmp(argv[1], "threads") == 0) return threads_main();
    std::mt19937_64 rng(20260111);
    auto U = [&](int lo, int hi) { return (int)std::uniform_int_distribution<int>(lo, hi)(rng); };
    Plan p;  // reused across calls, like the handle's
    for (int trial = 0; trial < 3000; ++trial) {
        const int64_t K = U(0, 60);
        const bool uni = U(0, 3) == 0;
        std::vector<int32_t> m(K), n(K), kind(K);
        for (int64_t k = 0; k < K; ++k) {
            kind[k] = U(0, 4) == 0 ? 1 : 0;
            n[k] = U(1, 300);
            m[k] = kind[k] ? 0 : U(1, 300);
        }
        if (uni)
            for (int64_t k = 1; k < K; ++k) m[k] = m[0], n[k] = n[0], kind[k] = kind[0];
        // planted errors (only in the entries the planner reads)
        const int64_t nread = uni ? (K > 0 ? 1 : 0) : K;
        int planted = 0;
        int64_t bad_k = -1;
        if (nread > 0 && U(0, 4) == 0) {
            bad_k = U(0, (int)nread - 1);
            planted = U(1, 4);
            if (planted == 1) kind[bad_k] = 2;
            if (planted == 2) kind[bad_k] = 0, m[bad_k] = 0;
            if (planted == 3) kind[bad_k] = 0, m[bad_k] = 2047;
            if (planted == 4) kind[bad_k] = 1, m[bad_k] = 3;
        }
        // offsets: packed (NULL), gapped increasing, or permuted
        const int mode = U(0, 2);
        std::vector<int64_t> ao(K), ro(K), co(K);
        std::vector<int64_t> perm(K);
        for (int64_t k = 0; k < K; ++k) perm[k] = k;
        if (mode == 2) std::shuffle(perm.begin(), perm.end(), rng);
        int64_t a = 0, r = 0, c = 0;
        for (int64_t q = 0; q < K; ++q) {
            const int64_t k = perm[q];
            if (mode) a += U(0, 9), r += U(0, 5), c += U(0, 5);
            ao[k] = a, ro[k] = r, co[k] = c;
            a += (int64_t)m[k] * n[k], r += m[k], c += n[k];
        }
        PlanIn in;
        in.count = K;
        in.uniform = uni;
        in.m = m.data();
        in.n = n.data();
        in.kind = kind.data();
        if (mode && !uni) in.a_off = ao.data(), in.row_off = ro.data(), in.col_off = co.data();
        in.has_A = in.has_b = in.has_sense = in.has_c = in.has_l = in.has_u = true;
        in.variants = kShapes;
        in.nreg = (int)(sizeof kShapes / sizeof kShapes[0]);
        in.force = U(0, 5) == 0 ? U(-2, in.nreg - 1) : -1;
        const int rc = plan_batch(in, p);
        if (planted) {
            const int want = planted == 3 ? PLAN_ERR_TOO_LARGE : PLAN_ERR_ARG;
            // an earlier invalid entry cannot exist (only one was planted)
            CHECK(rc == want, "trial %d planted %d at %lld: rc %d (%s)", trial, planted, (long long)bad_k, rc,
                  p.msg.c_str());
            char tag[32];
            std::snprintf(tag, sizeof tag, "LP %lld:", (long long)bad_k);
            CHECK(p.msg.find(tag) != std::string::npos, "trial %d: message '%s' names LP %lld", trial,
                  p.msg.c_str(), (long long)bad_k);
            continue;
        }
        CHECK(rc == PLAN_OK, "trial %d: rc %d (%s)", trial, rc, p.msg.c_str());
        if (rc != PLAN_OK) continue;
        // extents: every LP's ranges lie inside them, and some LP reaches each
        int64_t end_a = 0, end_r = 0, end_c = 0, slot = 0, simplex = 0, boxes = 0;
        std::set<int64_t> slots;
        for (int64_t k = 0; k < K; ++k) {
            const int64_t ak = uni ? k * m[0] * n[0] : (in.a_off ? ao[k] : -1);
            const int64_t rk = uni ? k * m[0] : (in.row_off ? ro[k] : -1);
            const int64_t ck = uni ? k * n[0] : (in.col_off ? co[k] : -1);
            if (!uni) {
                CHECK(p.a_off[k] >= 0 && p.row_off[k] >= 0 && p.col_off[k] >= 0, "trial %d: offsets", trial);
                if (in.a_off) CHECK(p.a_off[k] == ak && p.row_off[k] == rk && p.col_off[k] == ck, "trial %d", trial);
            }
            const int64_t a0 = uni ? ak : p.a_off[k], r0 = uni ? rk : p.row_off[k], c0 = uni ? ck : p.col_off[k];
            end_a = std::max(end_a, a0 + (int64_t)m[k] * n[k]);
            end_r = std::max(end_r, r0 + m[k]);
            end_c = std::max(end_c, c0 + n[k]);
            if (kind[k] == 0) {
                ++simplex;
                const int64_t ld = ((m[k] + 2 + 15) / 16) * 16;
                CHECK(ld >= m[k] + 2 && ld % 16 == 0, "ld");
                slots.insert(ld * (n[k] + m[k] + 1));
            } else {
                ++boxes;
            }
        }
        CHECK(p.tot_a == end_a && p.tot_m == end_r && p.tot_n == end_c, "trial %d: extents %lld %lld %lld vs %lld %lld %lld",
              trial, (long long)p.tot_a, (long long)p.tot_m, (long long)p.tot_n, (long long)end_a, (long long)end_r,
              (long long)end_c);
        if (!uni && !in.a_off) {
            // packed: the ranges tile [0, extent) without gaps or overlap
            int64_t sa = 0, sr = 0, sc = 0;
            for (int64_t k = 0; k < K; ++k) sa += (int64_t)m[k] * n[k], sr += m[k], sc += n[k];
            CHECK(sa == p.tot_a && sr == p.tot_m && sc == p.tot_n, "trial %d: packed extents", trial);
        }
        CHECK(p.any_simplex == (simplex > 0) && p.any_box == (boxes > 0), "trial %d: kinds", trial);
        CHECK(p.n_box == boxes, "trial %d: boxes", trial);
        if (simplex) CHECK(slots.count(p.max_slot) && p.max_slot == *slots.rbegin(), "trial %d: slot", trial);
        CHECK(p.n_may_stream >= 0 && p.n_may_stream <= simplex, "trial %d: may stream %lld of %lld", trial,
              (long long)p.n_may_stream, (long long)simplex);
        if (in.force == -2) CHECK(p.n_may_stream == simplex && (simplex == 0 || p.gm_deep), "trial %d: -2", trial);
    }
    // a shared box: every hyperbox LP must have the same n
    {
        std::vector<int32_t> m = {0, 3, 0, 0}, n = {5, 4, 5, 6}, kind = {1, 0, 1, 1};
        PlanIn in;
        in.count = 4;
        in.shared_box = true;
        in.m = m.data(), in.n = n.data(), in.kind = kind.data();
        in.has_A = in.has_b = in.has_sense = in.has_c = in.has_l = in.has_u = true;
        CHECK(plan_batch(in, p) == PLAN_ERR_ARG && p.msg.find("LP 3:") != std::string::npos, "shared box: %s",
              p.msg.c_str());
        n[3] = 5;
        CHECK(plan_batch(in, p) == PLAN_OK && p.box_n == 5, "shared box ok");
        in.has_l = false;
        CHECK(plan_batch(in, p) == PLAN_ERR_ARG, "missing l");
    }
    // copy runs of host-resident pieces
    std::vector<int64_t> order;
    std::vector<CopyRun> runs;
    for (int trial = 0; trial < 3000; ++trial) {
        const int64_t K = U(1, 80);
        std::vector<int32_t> len(K);
        std::vector<int64_t> off(K), perm(K);
        for (int64_t k = 0; k < K; ++k) len[k] = U(0, 7), perm[k] = k;
        if (U(0, 1)) std::shuffle(perm.begin(), perm.end(), rng);
        int64_t pos = 0;
        for (int64_t q = 0; q < K; ++q) {
            pos += U(0, 1) ? U(0, 4) : 0;
            off[perm[q]] = pos;
            pos += len[perm[q]];
        }
        const int64_t k0 = U(0, (int)K - 1), k1 = U((int)k0 + 1, (int)K);
        int64_t lo = INT64_MAX;
        for (int64_t k = k0; k < k1; ++k) lo = std::min(lo, off[k]);
        copy_runs(off, len, k0, k1, lo, order, runs);
        std::set<int64_t> want, got;
        for (int64_t k = k0; k < k1; ++k)
            for (int i = 0; i < len[k]; ++i) want.insert(off[k] + i);
        int64_t prev_end = -1;
        for (const CopyRun& r : runs) {
            CHECK(r.len > 0 && r.src == r.dst - lo && r.src >= 0, "trial %d: run", trial);
            CHECK(r.dst > prev_end, "trial %d: runs sorted and separated", trial);
            prev_end = r.dst + r.len - 1;
            for (int64_t i = 0; i < r.len; ++i) CHECK(got.insert(r.dst + i).second, "trial %d: overlap", trial);
        }
        CHECK(got == want, "trial %d: runs cover %zu positions, the piece's LPs %zu", trial, got.size(), want.size());
    }
    // chunk capacity (Eq. 5): the largest count that fits, never more than the batch
    for (int trial = 0; trial < 100000; ++trial) {
        const uint64_t limit = (uint64_t)U(0, 1 << 20), fixed = (uint64_t)U(0, 1 << 20), per = (uint64_t)U(0, 64);
        const int64_t K = U(0, 100000);
        const int64_t cap = chunk_capacity(limit, fixed, per, K);
        CHECK(cap >= 0 && cap <= K, "cap range");
        if (cap > 0) CHECK(fixed + (uint64_t)cap * per <= limit, "fits");
        if (cap < K && per > 0 && fixed <= limit)
            CHECK(fixed + (uint64_t)(cap + 1) * per > limit, "largest (limit %llu fixed %llu per %llu K %lld cap %lld)",
                  (unsigned long long)limit, (unsigned long long)fixed, (unsigned long long)per, (long long)K,
                  (long long)cap);
    }
    std::printf("host plan checks: %d failures\n", failures);
    return failures ? 1 : 0;
}
