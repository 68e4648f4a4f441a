// Host planning of batched launches: wave tasks, pairing, splitting of long
// lists, longest-first order and the task sublists (see plan_tasks), and the
// task lists of the table adjoint.  Plain C++: no HIP types, so the planner
// is also built on its own for host-side checks.
#include "planner.h"

#include <algorithm>
#include <string>
#include <vector>

namespace pgh {
namespace {

int fail_msg(std::string &err, int code, const std::string &msg)
{
    err = msg;
    return code;
}

// Orders idx stably by key(idx) (descending if asked): a counting sort when
// the keys are small non-negative integers (list lengths, wave-iterations),
// else a comparison sort.
template <class Key>
void stable_order(std::vector<int> &idx, Key key, bool descending, std::vector<int> &start,
                  std::vector<int> &out)
{
    long long kmax = 0;
    bool small = true;
    for (int k : idx) {
        const long long v = key(k);
        if (v < 0 || v > (1LL << 22)) {
            small = false;
            break;
        }
        kmax = std::max(kmax, v);
    }
    if (!small) {
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) {
            return descending ? key(a) > key(b) : key(a) < key(b);
        });
        return;
    }
    start.assign((size_t)kmax + 2, 0);
    for (int k : idx) {
        const long long v = key(k);
        ++start[(size_t)(descending ? kmax - v : v) + 1];
    }
    for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
    out.resize(idx.size());
    for (int k : idx) {
        const long long v = key(k);
        out[(size_t)start[(size_t)(descending ? kmax - v : v)]++] = k;
    }
    idx.swap(out);
}

// A chunk of at most 64 i-particles of one item (js lanes per i-particle).
struct Chunk {
    int i_off, n_i, j_off, n_j, js;
};

// A wave's work before splitting: one chunk, or two that share the wave.
struct Work {
    int a, b;  // chunk indices; b < 0: a single chunk
};

// The planner's temporaries, kept between calls on a host thread: plans of
// 10^5 tasks are rebuilt at every tree walk, and fresh vectors of that size
// cost more in first-touch page faults than the planning itself.
struct Scratch {
    std::vector<int> order, cand, idx, so_start, so_out;
    std::vector<Chunk> chunks;
    std::vector<Work> work;
    std::vector<Task> tasks;
    std::vector<long long> cost, c_it;
    std::vector<char> taken, c_taken;
    std::vector<int> c_ni, c_nj;
    std::vector<size_t> next_small;
};

Scratch &scratch()
{
    static thread_local Scratch s;
    return s;
}

}  // namespace

int plan_tasks(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               HostPlan &out, std::string &err)
{
    if (n_items < 0 || ni_total < 0 || nj_total < 0)
        return fail_msg(err, PGH_EINVAL, "counts must be >= 0");
    if (n_items > 0 && !items) return fail_msg(err, PGH_EINVAL, "NULL item array");
    Scratch &S = scratch();
    // ranges and disjointness of the i-groups
    std::vector<int> &order = S.order;
    order.clear();
    long long inter = 0;
    for (int t = 0; t < n_items; ++t) {
        const pgh_item &it = items[t];
        if (it.i_off < 0 || it.n_i < 0 || it.j_off < 0 || it.n_j < 0)
            return fail_msg(err, PGH_EINVAL, "item " + std::to_string(t) + " has a negative field");
        if ((long long)it.i_off + it.n_i > ni_total || (long long)it.j_off + it.n_j > nj_total)
            return fail_msg(err, PGH_ERANGE, "item " + std::to_string(t) + " exceeds the arrays");
        if (it.n_i > 0) order.push_back(t);
        inter += (long long)it.n_i * it.n_j;
    }
    std::sort(order.begin(), order.end(),
              [&](int a, int b) { return items[a].i_off < items[b].i_off; });
    for (size_t k = 1; k < order.size(); ++k) {
        const pgh_item &p0 = items[order[k - 1]], &p1 = items[order[k]];
        if (p1.i_off < p0.i_off + p0.n_i)
            return fail_msg(err, PGH_EINVAL, "i-ranges of items " + std::to_string(order[k - 1]) +
                                           " and " + std::to_string(order[k]) + " overlap");
    }

    // Wave tasks: chunks of <= 64 i-particles; a chunk of <= 32 (<= 16) runs
    // js = 2 (4) lanes per i-particle.  When chunks of 64 fill less than half
    // of the waves the device holds (a small plan), the groups are cut into
    // chunks of 32 or 16 instead: more waves to hide latency, each lane's
    // j-list shorter, and no partial sums (the lanes of an i-particle are
    // added inside the wave).
    waves = std::max(1, waves);
    int csize = 64;
    for (;;) {
        long long n = 0;
        for (int t : order) n += (items[t].n_i + csize - 1) / csize;
        if (n >= waves || csize == 16) break;
        csize /= 2;
    }
    std::vector<Chunk> &chunks = S.chunks;
    chunks.clear();
    long long total = 0;  // wave-iterations
    for (int t : order) {
        const pgh_item &it = items[t];
        for (int s0 = 0; s0 < it.n_i; s0 += csize) {
            const int n = std::min(csize, it.n_i - s0);
            const int js = n <= 16 ? 4 : (n <= 32 ? 2 : 1);
            chunks.push_back({it.i_off + s0, n, it.j_off, it.n_j, js});
            total += std::max(1LL, (long long)(it.n_j + js - 1) / js);
        }
    }
    // Cut j-lists longer than an eighth of the average work of a resident
    // wave, so each wave takes several tasks and the longest-first queue
    // ends with short ones.  (Equal tasks of half a wave's work leave the
    // last round of the queue mostly idle whenever the task count is just
    // above a multiple of the wave count.)
    const long long part_iters = std::max(512LL, (total / waves / 8 + 63) / 64 * 64);
    std::vector<Task> &tasks = S.tasks;
    std::vector<long long> &cost = S.cost;
    tasks.clear();
    cost.clear();
    std::vector<SplitChunk> &split = out.split;
    split.clear();
    int n_slots = 0;
    // Pair partly filled chunks: in order of j-list length, each takes the
    // first later one (within a short window) whose i-particles fit beside
    // its own in 64 lanes, when one wavefront running the longer list costs
    // fewer lane-iterations than the two apart.  A pair is cut along j like
    // any long list (both lists at the same offsets).
    std::vector<Work> &work = S.work;
    work.clear();
    {
        auto lane_iters = [](const Chunk &ch) {
            return 64LL * std::max(1LL, (long long)(ch.n_j + ch.js - 1) / ch.js);
        };
        std::vector<char> &taken = S.taken;
        taken.assign(chunks.size(), 0);
        std::vector<int> &cand = S.cand;
        cand.clear();
        for (size_t k = 0; k < chunks.size(); ++k)
            if (chunks[k].n_i < 64 && chunks[k].n_j > 0) cand.push_back((int)k);
        stable_order(cand, [&](int k) { return (long long)chunks[k].n_j; }, false, S.so_start,
                     S.so_out);
        // the scan reads candidates in this order: keep their fields contiguous
        const size_t nc = cand.size();
        std::vector<int> &c_ni = S.c_ni, &c_nj = S.c_nj;
        std::vector<long long> &c_it = S.c_it;
        std::vector<char> &c_taken = S.c_taken;
        c_ni.resize(nc);
        c_nj.resize(nc);
        c_it.resize(nc);
        c_taken.assign(nc, 0);
        for (size_t u = 0; u < nc; ++u) {
            const Chunk &ch = chunks[cand[u]];
            c_ni[u] = ch.n_i;
            c_nj[u] = ch.n_j;
            c_it[u] = lane_iters(ch);
        }
        // beside a chunk of more than 32 only one of at most 31 fits: such
        // chunks scan the later small ones only (next_small skips the rest)
        std::vector<size_t> &next_small = S.next_small;
        next_small.assign(nc + 1, nc);
        for (size_t v = nc; v-- > 0;) next_small[v] = c_ni[v] <= 31 ? v : next_small[v + 1];
        constexpr size_t kWindow = 64;
        for (size_t u = 0; u < nc; ++u) {
            if (c_taken[u]) continue;
            const int room = 64 - c_ni[u];
            const size_t v_end = std::min(nc, u + 1 + kWindow);
            const bool big = room <= 31;
            for (size_t v = big ? next_small[u + 1] : u + 1; v < v_end;
                 v = big ? next_small[v + 1] : v + 1) {
                if (c_taken[v] || c_ni[v] > room) continue;
                if (64LL * std::max(c_nj[u], c_nj[v]) >= c_it[u] + c_it[v]) continue;
                c_taken[u] = c_taken[v] = 1;
                taken[cand[u]] = taken[cand[v]] = 1;
                work.push_back({cand[u], cand[v]});
                break;
            }
        }
        for (size_t k = 0; k < chunks.size(); ++k)
            if (!taken[k]) work.push_back({(int)k, -1});
    }
    static const Chunk kNone{0, 0, 0, 0, 1};
    for (const Work &wk : work) {
        const Chunk &ch = chunks[wk.a];
        const bool pair = wk.b >= 0;
        struct {
            const Chunk &b;
        } w{pair ? chunks[wk.b] : kNone};
        const int js = pair ? 1 : ch.js;
        const int njm = pair ? std::max(ch.n_j, w.b.n_j) : ch.n_j;
        const long long iters = (njm + js - 1) / js;
        int parts = (int)std::max(1LL, (iters + part_iters - 1) / part_iters);
        long long per = njm;
        if (parts > 1) {
            // equal parts, each a multiple of 64 j-particles except the last
            per = (njm + parts - 1) / parts;
            per = (per + 63) / 64 * 64;
            parts = (int)((njm + per - 1) / per);
        }
        auto cut = [&](int n_j, int q) {
            return (int)std::max(0LL, std::min<long long>(per, n_j - q * per));
        };
        // where part q starts in a list of n_j entries (its end for the
        // empty parts of the shorter list of a pair)
        auto start = [&](int n_j, int q) { return (int)std::min<long long>((long long)q * per, n_j); };
        if (parts <= 1) {
            tasks.push_back({ch.i_off, ch.n_i, ch.j_off, ch.n_j, 0, 1, 0, w.b.i_off, w.b.n_i,
                             w.b.j_off, w.b.n_j, 0});
            cost.push_back(std::max(1LL, iters));
            continue;
        }
        for (int q = 0; q < parts; ++q) {
            const int nja = cut(ch.n_j, q), njb = pair ? cut(w.b.n_j, q) : 0;
            tasks.push_back({ch.i_off, ch.n_i, ch.j_off + start(ch.n_j, q), nja, q, parts, n_slots,
                             w.b.i_off, w.b.n_i, w.b.j_off + (pair ? start(w.b.n_j, q) : 0), njb,
                             0});
            cost.push_back((std::max(nja, njb) + js - 1) / js);
        }
        split.push_back({ch.i_off, ch.n_i, n_slots, parts, 0});
        if (pair) split.push_back({w.b.i_off, w.b.n_i, n_slots, parts, ch.n_i});
        n_slots += parts;
    }
    // longest tasks first
    std::vector<int> &idx = S.idx;
    idx.resize(tasks.size());
    for (size_t k = 0; k < idx.size(); ++k) idx[k] = (int)k;
    stable_order(idx, [&](int k) { return cost[k]; }, true, S.so_start, S.so_out);
    // Deal the longest-first list into nq sublists, a group of kBatchWaves
    // consecutive tasks at a time, round-robin: each sublist stays longest
    // first with an equal share of every size class, and workgroup b (which
    // serves sublist b mod nq) takes tasks 4b .. 4b+3 of the whole list in
    // its first round, one of similar length per SIMD.
    const int nq = (int)std::min<size_t>(
        kQueues, std::max<size_t>(1, (idx.size() + kBatchWaves - 1) / kBatchWaves));
    std::vector<Task> &sorted = out.tasks;
    sorted.clear();
    int *q_begin = out.q_begin;
    std::fill(q_begin, q_begin + kQueues + 1, 0);
    for (int q = 0; q < nq; ++q) {
        q_begin[q] = (int)sorted.size();
        for (size_t g0 = (size_t)q * kBatchWaves; g0 < idx.size(); g0 += (size_t)nq * kBatchWaves)
            for (size_t k = g0; k < std::min(idx.size(), g0 + kBatchWaves); ++k)
                sorted.push_back(tasks[idx[k]]);
    }
    q_begin[nq] = (int)sorted.size();

    out.nq = nq;
    out.n_slots = n_slots;
    out.interactions = inter;
    out.ordered.clear();
    out.ordered.reserve(order.size());
    for (int t : order) out.ordered.push_back(items[t]);
    return PGH_OK;
}

void plan_adjoint_tasks(const std::vector<pgh_item> &ordered, int waves, std::vector<Task> &out_j,
                        std::vector<Task> &out_i)
{
    const std::vector<pgh_item> &ord = ordered;
    waves = std::max(1, waves);
    // i-major tasks of the table adjoint (the i-side position gradient, its
    // own list independent of the forward's chunking): i-chunks of <= 64
    // against j-ranges of <= 512, added with atomics, so no partial sums
    std::vector<Task> &it_tasks = out_i;
    it_tasks.clear();
    for (const pgh_item &it : ord) {
        for (int s0 = 0; s0 < it.n_i; s0 += 64)
            for (int q0 = 0; q0 < it.n_j; q0 += 512)
                it_tasks.push_back({it.i_off + s0, std::min(64, it.n_i - s0), it.j_off + q0,
                                    std::min(512, it.n_j - q0), 0, 1, 0, 0, 0, 0, 0, 0});
    }
    std::stable_sort(it_tasks.begin(), it_tasks.end(), [](const Task &a, const Task &b) {
        return (long long)a.n_j * ((a.n_i + 15) / 16) > (long long)b.n_j * ((b.n_i + 15) / 16);
    });
    // j-major tasks of the table adjoint: chunks of <= 64 j-entries of a
    // list against its i-group (chunks of 32 or 16, 2 or 4 lanes per entry,
    // when chunks of 64 would fill less than half of the resident waves)
    int jc = 64;
    for (;;) {
        long long n = 0;
        for (const pgh_item &it : ord) n += (it.n_j + jc - 1) / jc;
        if (2 * n >= waves || jc == 16) break;
        jc /= 2;
    }
    std::vector<Task> &jt = out_j;
    jt.clear();
    for (const pgh_item &it : ord) {
        for (int s0 = 0; s0 < it.n_j; s0 += jc)
            jt.push_back({it.j_off + s0, std::min(jc, it.n_j - s0), it.i_off, it.n_i, 0, 1, 0, 0, 0,
                          0, 0, 0});
    }
    std::stable_sort(jt.begin(), jt.end(), [](const Task &a, const Task &b) { return a.n_j > b.n_j; });
}

}  // namespace pgh
