// Host-side checker of the batched-launch planner (built with AddressSanitizer
// and UndefinedBehaviorSanitizer by tests/test_planner_cpu.py).
//
// For random item sets of the shapes the library meets (tree-style groups,
// cell-grid lists, tiny groups, one giant list, empty groups and lists, items
// in any order with gaps between them) it builds plans for several device
// sizes, plain and packed, and checks what the batched kernels rely on:
//   * every (i, j) pair of every item is in exactly one task (a split list's
//     parts, and both chunks of a paired task, included), and every row of
//     an item with n_i > 0 is in some task, so each output row is written;
//   * tasks fit a wave (n_i <= 64; two paired chunks fit in 32 lane rows of
//     two i-particles each);
//   * split parts: each (slot, part) is used once, slots below n_slots, and
//     each split chunk's lanes fit in its slots;
//   * sublists: q_begin covers the tasks in order, at most 16 sublists, each
//     sublist longest first;
//   * the interaction count, and the error status of invalid items;
//   * the table adjoint's task lists cover every pair once.
// Prints "planner checks passed" and exits 0, or prints the first failure
// and exits 1.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "planner.h"

using namespace pgh;

namespace {

int failures = 0;
int compact_checked = 0;  // plans whose compact form was checked

void fail(const std::string &what)
{
    if (failures++ == 0) std::printf("FAIL: %s\n", what.c_str());
}

struct Span {
    long long a, b;  // [a, b)
};

// The j-intervals of every row, checked against each row's item.
bool check_cover(const std::vector<pgh_item> &items, int ni_total,
                 const std::vector<std::vector<Span>> &rows, const char *what)
{
    std::vector<int> owner(ni_total, -1);
    for (size_t t = 0; t < items.size(); ++t)
        for (int r = items[t].i_off; r < items[t].i_off + items[t].n_i; ++r) owner[r] = (int)t;
    for (int r = 0; r < ni_total; ++r) {
        std::vector<Span> v = rows[r];
        if (owner[r] < 0) {
            if (!v.empty()) {
                fail(std::string(what) + ": a row outside every item is in a task");
                return false;
            }
            continue;
        }
        const pgh_item &it = items[owner[r]];
        if (v.empty()) {
            fail(std::string(what) + ": row " + std::to_string(r) + " is in no task");
            return false;
        }
        std::sort(v.begin(), v.end(), [](const Span &x, const Span &y) {
            return x.a < y.a || (x.a == y.a && x.b < y.b);
        });
        long long at = it.j_off;
        for (const Span &s : v) {
            if (s.a == s.b) continue;  // an empty part (allowed: a list of length 0)
            if (s.a != at) {
                fail(std::string(what) + ": row " + std::to_string(r) + " has a gap or overlap at j " +
                     std::to_string(at));
                return false;
            }
            at = s.b;
        }
        if (at != (long long)it.j_off + it.n_j) {
            fail(std::string(what) + ": row " + std::to_string(r) + " misses the end of its list");
            return false;
        }
    }
    return true;
}

// The compact form of the plan (plan_descs) expanded here as the device
// expands it (every task from its entry, a stable sort by kmax - cost, the
// dealt positions) gives the same tasks, split chunks and sublists.
void check_compact(const std::vector<pgh_item> &items, int ni_total, int nj_total, int waves,
                   const HostPlan &hp, const std::vector<Task> &T, const char *what)
{
    DescPlan dp;
    std::string err;
    const int st = plan_descs(items.data(), (int)items.size(), ni_total, nj_total, waves, dp, err);
    if (st == kPlanOnHost) return;
    if (st != PGH_OK) {
        fail(std::string(what) + ": plan_descs failed: " + err);
        return;
    }
    if (dp.n_tasks != hp.n_tasks || dp.n_slots != hp.n_slots ||
        dp.n_split != (int)hp.split.size() || dp.nq != hp.nq ||
        !std::equal(dp.q_begin, dp.q_begin + kQueues + 1, hp.q_begin) ||
        dp.interactions != hp.interactions) {
        fail(std::string(what) + ": compact plan counts differ");
        return;
    }
    const int n = dp.n_tasks;
    std::vector<Task> raw(n);
    std::vector<unsigned> key(n);
    std::vector<SplitChunk> split(dp.n_split, SplitChunk{-1, -1, -1, -1, -1});
    size_t d = 0;
    for (int t = 0; t < n; ++t) {
        while (d + 1 < dp.desc.size() && dp.desc[d + 1].task0 <= t) ++d;
        int cost = 0, ns = 0, at = 0;
        SplitChunk sc[2];
        raw[t] = desc_task(dp.desc[d], t - dp.desc[d].task0, dp.part_iters, &cost, sc, &ns, &at);
        if (cost < 1 || (unsigned)cost > dp.kmax) {
            fail(std::string(what) + ": compact plan cost outside [1, kmax]");
            return;
        }
        key[t] = dp.kmax - (unsigned)cost;
        for (int k = 0; k < ns; ++k) {
            if (at + k < 0 || at + k >= dp.n_split) {
                fail(std::string(what) + ": compact plan split index out of range");
                return;
            }
            split[at + k] = sc[k];
        }
    }
    std::vector<int> idx(n);
    for (int t = 0; t < n; ++t) idx[t] = t;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return key[a] < key[b]; });
    std::vector<Task> dealt(n);
    for (int r = 0; r < n; ++r) dealt[dealt_position(r, dp.nq, dp.q_begin)] = raw[idx[r]];
    auto same_task = [](const Task &a, const Task &b) {
        return a.i_off == b.i_off && a.n_i == b.n_i && a.j_off == b.j_off && a.n_j == b.n_j &&
               a.part == b.part && a.n_parts == b.n_parts && a.slot == b.slot &&
               a.i_off2 == b.i_off2 && a.n_i2 == b.n_i2 && a.j_off2 == b.j_off2 &&
               a.n_j2 == b.n_j2;
    };
    for (int k = 0; k < n; ++k)
        if (!same_task(dealt[k], T[k])) {
            fail(std::string(what) + ": compact plan task " + std::to_string(k) + " differs");
            return;
        }
    for (size_t k = 0; k < split.size(); ++k) {
        const SplitChunk &a = split[k], &b = hp.split[k];
        if (a.i_off != b.i_off || a.n_i != b.n_i || a.slot != b.slot || a.n_parts != b.n_parts ||
            a.lane0 != b.lane0) {
            fail(std::string(what) + ": compact plan split chunk " + std::to_string(k) + " differs");
            return;
        }
    }
    ++compact_checked;
}

long long task_cost(const Task &t)
{
    const bool paired = t.n_i2 > 0;
    const int js = paired ? 1 : (t.n_i <= 16 ? 4 : (t.n_i <= 32 ? 2 : 1));
    const long long nj = paired ? std::max(t.n_j, t.n_j2) : t.n_j;
    return std::max(1LL, (nj + js - 1) / js);
}

void check_plan_one(const std::vector<pgh_item> &items, int ni_total, int nj_total, int waves,
                    const char *what, bool pack)
{
    HostPlan hp;
    std::string err;
    const int st =
        plan_tasks(items.data(), (int)items.size(), ni_total, nj_total, waves, hp, err, pack);
    if (st != PGH_OK) {
        fail(std::string(what) + ": plan_tasks failed: " + err);
        return;
    }
    long long inter = 0;
    for (const pgh_item &it : items) inter += (long long)it.n_i * it.n_j;
    if (inter != hp.interactions) fail(std::string(what) + ": interaction count");
    std::vector<Task> T(hp.n_tasks);
    write_tasks(hp, T.data());
    if (!T.empty()) {
        if (hp.nq < 1 || hp.nq > kQueues) fail(std::string(what) + ": sublist count");
        if (hp.q_begin[0] != 0 || hp.q_begin[hp.nq] != (int)T.size())
            fail(std::string(what) + ": sublists do not cover the tasks");
        for (int q = 0; q < hp.nq; ++q) {
            if (hp.q_begin[q] > hp.q_begin[q + 1]) fail(std::string(what) + ": sublist order");
            for (int k = hp.q_begin[q] + 1; k < hp.q_begin[q + 1]; ++k)
                if (task_cost(T[k]) > task_cost(T[k - 1]))
                    fail(std::string(what) + ": sublist " + std::to_string(q) + " not longest first");
        }
    }
    std::vector<std::vector<Span>> rows(ni_total);
    std::vector<int> used;  // (slot, part) uses
    for (const Task &t : T) {
        if (t.n_i < 1 || t.n_i > 64) fail(std::string(what) + ": task n_i out of [1, 64]");
        if (t.n_i2 < 0 || t.n_i + t.n_i2 > 64 || (t.n_i + 1) / 2 + (t.n_i2 + 1) / 2 > 32)
            fail(std::string(what) + ": paired chunks exceed 32 rows of two lanes");
        if (t.n_parts < 1 || t.part < 0 || t.part >= t.n_parts) fail(std::string(what) + ": part fields");
        if (t.i_off < 0 || t.i_off + t.n_i > ni_total || t.j_off < 0 || t.j_off + t.n_j > nj_total)
            fail(std::string(what) + ": task outside the arrays");
        if (t.n_i2 > 0 && (t.i_off2 < 0 || t.i_off2 + t.n_i2 > ni_total || t.j_off2 < 0 ||
                           t.j_off2 + t.n_j2 > nj_total))
            fail(std::string(what) + ": paired chunk outside the arrays");
        if (failures) return;
        for (int r = t.i_off; r < t.i_off + t.n_i; ++r) rows[r].push_back({t.j_off, (long long)t.j_off + t.n_j});
        for (int r = t.i_off2; r < t.i_off2 + t.n_i2; ++r)
            rows[r].push_back({t.j_off2, (long long)t.j_off2 + t.n_j2});
        if (t.n_parts > 1) {
            const int slot = t.slot + t.part;
            if (slot < 0 || slot >= hp.n_slots) fail(std::string(what) + ": slot out of range");
            used.push_back(slot);
        }
    }
    std::sort(used.begin(), used.end());
    if (std::adjacent_find(used.begin(), used.end()) != used.end())
        fail(std::string(what) + ": a partial-sum slot is written by two tasks");
    for (const SplitChunk &c : hp.split)
        if (c.lane0 < 0 || c.lane0 + c.n_i > 64 || c.slot < 0 || c.slot + c.n_parts > hp.n_slots)
            fail(std::string(what) + ": split chunk outside its slots");
    if (failures) return;
    check_cover(items, ni_total, rows, what);
    // the compact form holds the unpacked cut only
    if (!pack) check_compact(items, ni_total, nj_total, waves, hp, T, what);
    // the table adjoint's tasks: j-major (j-chunk against the item's i-range)
    // and i-major (i-chunk against a j-range) each cover every pair once
    std::vector<Task> jt, it;
    plan_adjoint_tasks(hp.ordered, waves, jt, it);
    std::vector<std::vector<Span>> rows_j(ni_total), rows_i(ni_total);
    for (const Task &t : jt) {  // fields: j_off, n_j (chunk) in i_off / n_i slots
        if (t.n_i < 1 || t.n_i > 64) fail(std::string(what) + ": adjoint j-chunk size");
        for (int r = t.j_off; r < t.j_off + t.n_j; ++r)
            rows_j[r].push_back({t.i_off, (long long)t.i_off + t.n_i});
    }
    for (const Task &t : it) {
        if (t.n_i < 1 || t.n_i > 64) fail(std::string(what) + ": adjoint i-chunk size");
        for (int r = t.i_off; r < t.i_off + t.n_i; ++r)
            rows_i[r].push_back({t.j_off, (long long)t.j_off + t.n_j});
    }
    if (failures) return;
    // rows with n_j = 0 have no adjoint work: compare against the items
    // that have a j-list
    std::vector<pgh_item> with_j;
    for (const pgh_item &x : items)
        if (x.n_i > 0 && x.n_j > 0) with_j.push_back(x);
    check_cover(with_j, ni_total, rows_i, "adjoint i-major");
    check_cover(with_j, ni_total, rows_j, "adjoint j-major");
}

// Every check, on the plain plan and on the packed one (chunks of 64 that
// take the next item's first i-particles into their empty rows).
void check_plan(const std::vector<pgh_item> &items, int ni_total, int nj_total, int waves,
                const char *what)
{
    check_plan_one(items, ni_total, nj_total, waves, what, false);
    check_plan_one(items, ni_total, nj_total, waves, (std::string(what) + ", packed").c_str(), true);
}

// Items over a permutation of disjoint i-ranges with gaps; n_i and n_j from
// the given generators.
template <class NI, class NJ>
std::vector<pgh_item> make_items(std::mt19937 &rng, int n_items, NI ni, NJ nj, int *ni_total,
                                 int *nj_total)
{
    std::vector<pgh_item> v;
    int i_at = 0, j_at = 0;
    for (int k = 0; k < n_items; ++k) {
        const int gap = (rng() % 7 == 0) ? (int)(rng() % 5) : 0;
        i_at += gap;
        const int a = ni(), b = nj();
        v.push_back({i_at, a, j_at, b});
        i_at += a;
        j_at += b;
    }
    std::shuffle(v.begin(), v.end(), rng);
    *ni_total = i_at + 3;
    *nj_total = j_at;
    return v;
}

}  // namespace

int main()
{
    std::mt19937 rng(12345);
    auto U = [&](int lo, int hi) { return lo + (int)(rng() % (unsigned)(hi - lo + 1)); };
    const int wave_counts[] = {1, 100, 2048, 8192};
    for (int rep = 0; rep < 3 && !failures; ++rep) {
        for (int waves : wave_counts) {
            int ni_total = 0, nj_total = 0;
            std::vector<pgh_item> items;
            items = make_items(rng, U(1, 400), [&] { return U(1, 300); },
                               [&] { return rng() % 9 == 0 ? U(0, 30000) : U(0, 3000); }, &ni_total,
                               &nj_total);
            check_plan(items, ni_total, nj_total, waves, "tree-style");
            std::poisson_distribution<int> pois(64);
            items = make_items(rng, U(64, 600), [&] { return std::max(0, pois(rng)); },
                               [&] { return U(150, 300); }, &ni_total, &nj_total);
            check_plan(items, ni_total, nj_total, waves, "cell-style");
            items = make_items(rng, U(1, 40), [&] { return U(0, 20); }, [&] { return U(0, 40); },
                               &ni_total, &nj_total);
            check_plan(items, ni_total, nj_total, waves, "tiny");
            items = make_items(rng, 1, [&] { return 5000; }, [&] { return 100000; }, &ni_total,
                               &nj_total);
            check_plan(items, ni_total, nj_total, waves, "giant");
            check_plan({}, 10, 10, waves, "empty");
        }
    }
    // tree-code sized item sets (groups of up to 1024, long lists, a few very
    // long ones): chunks of 64 fill the device, so their compact form is used
    for (int rep = 0; rep < 3 && !failures; ++rep) {
        for (int waves : {1024, 4096}) {
            int ni_total = 0, nj_total = 0;
            std::vector<pgh_item> items = make_items(
                rng, U(300, 900), [&] { return rng() % 5 == 0 ? U(1, 63) : U(1, 1024); },
                [&] { return rng() % 50 == 0 ? U(20000, 200000) : U(0, 6000); }, &ni_total,
                &nj_total);
            check_plan(items, ni_total, nj_total, waves, "tree-code");
        }
    }
    // invalid items: overlapping i-ranges, out of range, negative fields
    {
        HostPlan hp;
        std::string err;
        const std::vector<pgh_item> overlap = {{0, 10, 0, 5}, {5, 10, 5, 5}};
        if (plan_tasks(overlap.data(), 2, 20, 10, 2048, hp, err) != PGH_EINVAL)
            fail("overlapping i-ranges accepted");
        const std::vector<pgh_item> beyond = {{0, 10, 0, 11}};
        if (plan_tasks(beyond.data(), 1, 10, 10, 2048, hp, err) != PGH_ERANGE)
            fail("a j-range beyond the arrays accepted");
        const std::vector<pgh_item> negative = {{0, -1, 0, 1}};
        if (plan_tasks(negative.data(), 1, 10, 10, 2048, hp, err) != PGH_EINVAL)
            fail("a negative field accepted");
        if (plan_tasks(nullptr, 3, 10, 10, 2048, hp, err) != PGH_EINVAL) fail("NULL items accepted");
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    if (compact_checked < 20) {
        std::printf("only %d compact plans checked\n", compact_checked);
        return 1;
    }
    std::printf("planner checks passed (%d compact plans)\n", compact_checked);
    return 0;
}
