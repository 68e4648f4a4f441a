// Host planning of batched launches: wave tasks, pairing, splitting of long
// lists, longest-first order and the task sublists (plan_tasks), the compact
// form of the same plan whose tasks the device expands (plan_descs), and the
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

// The planner's temporaries, kept between calls on a host thread: plans of
// 10^5 tasks are rebuilt at every tree walk, and fresh vectors of that size
// cost more in first-touch page faults than the planning itself.
struct Scratch {
    std::vector<int> order, cand, so_start, so_out;
    std::vector<PlanRef> refs;
    std::vector<int> cost;
    std::vector<long long> c_it;
    std::vector<char> taken;
    std::vector<int> c_ni, c_nj;
    std::vector<unsigned long long> fits, big, used;  // bit sets over the candidates
    std::vector<std::pair<int, int>> pairs, packed;
};

Scratch &scratch()
{
    static thread_local Scratch s;
    return s;
}

// Checks the items (non-negative fields, inside the arrays, disjoint
// i-ranges), and lists those with n_i > 0 by i_off in `order` and `ordered`.
int validate_items(const pgh_item *items, int n_items, int ni_total, int nj_total,
                   std::vector<int> &order, std::vector<pgh_item> &ordered, long long *inter,
                   std::string &err)
{
    if (n_items < 0 || ni_total < 0 || nj_total < 0)
        return fail_msg(err, PGH_EINVAL, "counts must be >= 0");
    if (n_items > 0 && !items) return fail_msg(err, PGH_EINVAL, "NULL item array");
    order.clear();
    *inter = 0;
    bool sorted = true;
    for (int t = 0; t < n_items; ++t) {
        const pgh_item &it = items[t];
        if (it.i_off < 0 || it.n_i < 0 || it.j_off < 0 || it.n_j < 0)
            return fail_msg(err, PGH_EINVAL, "item " + std::to_string(t) + " has a negative field");
        if ((long long)it.i_off + it.n_i > ni_total || (long long)it.j_off + it.n_j > nj_total)
            return fail_msg(err, PGH_ERANGE, "item " + std::to_string(t) + " exceeds the arrays");
        if (it.n_i > 0) {
            if (!order.empty() && it.i_off < items[order.back()].i_off) sorted = false;
            order.push_back(t);
        }
        *inter += (long long)it.n_i * it.n_j;
    }
    if (!sorted)
        std::sort(order.begin(), order.end(),
                  [&](int a, int b) { return items[a].i_off < items[b].i_off; });
    for (size_t k = 1; k < order.size(); ++k) {
        const pgh_item &p0 = items[order[k - 1]], &p1 = items[order[k]];
        if (p1.i_off < p0.i_off + p0.n_i)
            return fail_msg(err, PGH_EINVAL, "i-ranges of items " + std::to_string(order[k - 1]) +
                                           " and " + std::to_string(order[k]) + " overlap");
    }
    ordered.clear();
    ordered.reserve(order.size());
    for (int t : order) ordered.push_back(items[t]);
    return PGH_OK;
}

// Pairs partly filled chunks.  cand lists the candidates (chunks of fewer
// than 64 i-particles with a non-empty list) in chunk order, with their
// i-particle counts ni[k] and list lengths nj[k] (indexed by the values in
// cand).  In order of list length, each candidate takes the first later one
// (within a window of 64) whose i-particles fit beside its own in 32 lane
// rows of two (at most 64 i-particles, at most 62 when both counts are odd),
// when one wavefront running the longer list costs fewer lane-iterations
// than the two apart.  Appends the pairs (chunk indices, the earlier first)
// in the order they are formed.
template <class NI, class NJ>
void pair_chunks(Scratch &S, std::vector<int> &cand, NI ni, NJ nj,
                 std::vector<std::pair<int, int>> &pairs)
{
    pairs.clear();
    stable_order(cand, [&](int k) { return (long long)nj(k); }, false, S.so_start, S.so_out);
    const size_t nc = cand.size();
    std::vector<int> &c_ni = S.c_ni, &c_nj = S.c_nj;
    std::vector<long long> &c_it = S.c_it;
    c_ni.resize(nc);
    c_nj.resize(nc);
    c_it.resize(nc);
    for (size_t u = 0; u < nc; ++u) {
        c_ni[u] = ni(cand[u]);
        c_nj[u] = nj(cand[u]);
        c_it[u] = 64LL * std::max(1LL, lane_steps(c_nj[u], chunk_js(c_ni[u])));
    }
    // Bit sets over the candidates (in this order): fits[r] holds those of
    // at most r i-particles, big those of more than 32 (one lane each), used
    // those already paired.  A candidate's partners are then the set bits of
    // fits[room] & ~used in its window, in order.  Two chunks of at most 32
    // (two or four lanes each) can only gain by sharing when their lists
    // differ by at most one entry (rounding of the lane counts), so past
    // that point a small chunk looks at big ones only.
    const size_t nw = (nc + 63) / 64 + 1;
    std::vector<unsigned long long> &fits = S.fits, &big = S.big, &used = S.used;
    fits.assign(64 * nw, 0ULL);
    big.assign(nw, 0ULL);
    used.assign(nw, 0ULL);
    for (size_t u = 0; u < nc; ++u) {
        fits[(size_t)c_ni[u] * nw + u / 64] |= 1ULL << (u % 64);
        if (c_ni[u] > 32) big[u / 64] |= 1ULL << (u % 64);
    }
    for (int r = 1; r < 64; ++r)
        for (size_t w = 0; w < nw; ++w) fits[(size_t)r * nw + w] |= fits[(size_t)(r - 1) * nw + w];
    // the bits [from, from + len) of a set, len <= 64
    auto window = [&](const unsigned long long *set, size_t from, size_t len) {
        const size_t w = from / 64, sh = from % 64;
        unsigned long long m = set[w] >> sh;
        if (sh) m |= set[w + 1] << (64 - sh);
        return len < 64 ? m & ((1ULL << len) - 1) : m;
    };
    constexpr size_t kWindow = 64;
    for (size_t u = 0; u < nc; ++u) {
        if (used[u / 64] >> (u % 64) & 1) continue;
        const size_t from = u + 1, len = std::min(nc, u + 1 + kWindow) - from;
        if (len == 0) break;
        // two chunks share a wave when their i-particles fit in 32 lane rows
        // of two slots each (ceil(n_1 / 2) + ceil(n_2 / 2) <= 32), so a
        // kernel holding two i-particles per lane can run the pair as one
        // lane per i-particle can
        const int room = 64 - 2 * ((c_ni[u] + 1) / 2);
        unsigned long long m =
            window(&fits[(size_t)room * nw], from, len) & ~window(used.data(), from, len);
        if (c_ni[u] <= 32) {
            // small candidates only up to list length c_nj[u] + 1
            const size_t near =
                std::upper_bound(c_nj.begin() + from, c_nj.begin() + from + len,
                                 (long long)c_nj[u] + 1) -
                (c_nj.begin() + from);
            const unsigned long long head = near < 64 ? (1ULL << near) - 1 : ~0ULL;
            m &= head | window(big.data(), from, len);
        }
        for (; m; m &= m - 1) {
            const size_t v = from + (size_t)__builtin_ctzll(m);
            if (64LL * std::max(c_nj[u], c_nj[v]) >= c_it[u] + c_it[v]) continue;
            used[u / 64] |= 1ULL << (u % 64);
            used[v / 64] |= 1ULL << (v % 64);
            pairs.push_back({cand[u], cand[v]});
            break;
        }
    }
}

// Sublists of a plan of n tasks: their count and starts (q_begin[nq] = n).
// Sublist q holds the groups of kBatchWaves ranks g = q, q + nq, ...; only
// the last group of all may be partial.
int deal_layout(size_t n, int *q_begin)
{
    const int nq = (int)std::min<size_t>(kQueues, std::max<size_t>(1, (n + kBatchWaves - 1) / kBatchWaves));
    std::fill(q_begin, q_begin + kQueues + 1, 0);
    const size_t groups = (n + kBatchWaves - 1) / kBatchWaves;
    for (int q = 0; q < nq; ++q) {
        size_t size = (groups / nq + ((size_t)q < groups % nq ? 1 : 0)) * kBatchWaves;
        if (groups > 0 && (size_t)q == (groups - 1) % nq) size -= groups * kBatchWaves - n;
        q_begin[q + 1] = q_begin[q] + (int)size;
    }
    return nq;
}

// Part length of the lists: an eighth of the average work of a resident
// wave, so each wave takes several tasks and the longest-first queue ends
// with short ones.  (Equal tasks of half a wave's work leave the last round
// of the queue mostly idle whenever the task count is just above a multiple
// of the wave count.)
long long part_length(long long wave_iters, int waves)
{
    return std::max(512LL, (wave_iters / waves / 8 + 63) / 64 * 64);
}

}  // namespace

int plan_tasks(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               HostPlan &out, std::string &err, bool pack)
{
    Scratch &S = scratch();
    std::vector<int> &order = S.order;
    long long inter = 0;
    {
        const int st = validate_items(items, n_items, ni_total, nj_total, order, out.ordered,
                                      &inter, err);
        if (st) return st;
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
    std::vector<PlanChunk> &chunks = out.chunks;
    chunks.clear();
    long long total = 0;  // wave-iterations
    // Packing (chunks of 64 only): the rows an item leaves empty in its last
    // chunk are filled with the first i-particles of the next item, as a
    // paired task (each lane over its own item's list), whenever one wave
    // running the longer list costs fewer lane-iterations than the two
    // apart; the rest of the next item is cut after them.  The i-particles of
    // an item need no combining however they are cut, so a stream of groups
    // of about 64 becomes fewer and fuller tasks (4^3 cell lists of 262144
    // particles: 4196 tasks instead of 4920, 22.8 us per call instead of
    // 23.9).
    pack = pack && csize == 64;
    std::vector<std::pair<int, int>> &packed = S.packed;
    packed.clear();
    auto iters = [](int n, int nj) { return 64LL * std::max(1LL, lane_steps(nj, chunk_js(n))); };
    int open = -1;  // the previous item's partly filled last chunk, awaiting a partner
    for (int t : order) {
        const pgh_item &it = items[t];
        int s0 = 0;
        if (pack && open >= 0 && it.n_j > 0) {
            const PlanChunk &o = chunks[(size_t)open];
            // rows of two slots: the pair fits when ceil(n_1 / 2) + ceil(n_2 / 2) <= 32
            const int h = std::min(64 - 2 * ((o.n_i + 1) / 2), it.n_i);
            if (h > 0 && 64LL * std::max(o.n_j, it.n_j) < iters(o.n_i, o.n_j) + iters(h, it.n_j)) {
                chunks.push_back({it.i_off, h, it.j_off, it.n_j, chunk_js(h)});
                total += std::max(1LL, lane_steps(it.n_j, chunk_js(h)));
                packed.push_back({open, (int)chunks.size() - 1});
                s0 = h;
            }
        }
        open = -1;
        for (; s0 < it.n_i; s0 += csize) {
            const int n = std::min(csize, it.n_i - s0);
            const int js = chunk_js(n);
            chunks.push_back({it.i_off + s0, n, it.j_off, it.n_j, js});
            total += std::max(1LL, lane_steps(it.n_j, js));
            if (pack && n < 64 && it.n_j > 0) open = (int)chunks.size() - 1;
        }
    }
    const long long part_iters = part_length(total, waves);
    // add_work records a wave's work (chunk a, and chunk b sharing the wave,
    // or b < 0), its cut and its tasks with their costs
    std::vector<PlanWork> &work = out.work;
    work.clear();
    std::vector<PlanRef> &refs = S.refs;
    std::vector<int> &cost = S.cost;
    refs.clear();
    cost.clear();
    std::vector<SplitChunk> &split = out.split;
    split.clear();
    int n_slots = 0;
    auto add_work = [&](int a, int b) {
        const int w = (int)work.size();
        const PlanChunk &ch = chunks[a];
        const bool pair = b >= 0;
        const int njb = pair ? chunks[b].n_j : 0;
        const WorkCut c = cut_work(std::max(ch.n_j, njb), pair ? 1 : ch.js, part_iters);
        work.push_back({a, b, c.parts, c.per, c.parts > 1 ? n_slots : 0});
        for (int q = 0; q < c.parts; ++q) {
            refs.push_back({w, q});
            cost.push_back(work_task_cost(ch.n_i, ch.n_j, pair, njb, c, q));
        }
        if (c.parts > 1) {
            split.push_back({ch.i_off, ch.n_i, n_slots, c.parts, 0});
            if (pair) split.push_back({chunks[b].i_off, chunks[b].n_i, n_slots, c.parts, ch.n_i});
            n_slots += c.parts;
        }
    };
    // paired works first, in the order the pairs form, then every other
    // chunk in chunk order
    {
        if (pack) {
            S.pairs = packed;
        } else {
            std::vector<int> &cand = S.cand;
            cand.clear();
            for (size_t k = 0; k < chunks.size(); ++k)
                if (chunks[k].n_i < 64 && chunks[k].n_j > 0) cand.push_back((int)k);
            pair_chunks(S, cand, [&](int k) { return chunks[k].n_i; },
                        [&](int k) { return chunks[k].n_j; }, S.pairs);
        }
        std::vector<char> &taken = S.taken;
        taken.assign(chunks.size(), 0);
        for (const auto &pr : S.pairs) {
            taken[pr.first] = taken[pr.second] = 1;
            add_work(pr.first, pr.second);
        }
        for (size_t k = 0; k < chunks.size(); ++k)
            if (!taken[k]) add_work((int)k, -1);
    }
    // Longest tasks first, dealt into nq sublists a group of kBatchWaves
    // consecutive tasks at a time, round-robin: each sublist stays longest
    // first with an equal share of every size class, and workgroup b (which
    // serves sublist b mod nq) takes tasks 4b .. 4b+3 of the whole list in
    // its first round, one of similar length per SIMD.
    const size_t n = refs.size();
    if (n > (size_t)(1 << 30)) return fail_msg(err, PGH_ERANGE, "the plan exceeds 2^30 tasks");
    int *q_begin = out.q_begin;
    const int nq = deal_layout(n, q_begin);
    std::vector<PlanRef> &dealt = out.dealt;
    dealt.resize(n);
    int kmax = 0;
    for (int c : cost) kmax = std::max(kmax, c);
    if (kmax <= (1 << 22)) {
        // stable counting sort, longest first, scattered straight to the
        // dealt positions
        std::vector<int> &start = S.so_start;
        start.assign((size_t)kmax + 2, 0);
        for (int c : cost) ++start[(size_t)(kmax - c) + 1];
        for (size_t b = 1; b < start.size(); ++b) start[b] += start[b - 1];
        for (size_t k = 0; k < n; ++k)
            dealt[dealt_position(start[(size_t)(kmax - cost[k])]++, nq, q_begin)] = refs[k];
    } else {
        std::vector<int> &idx = S.order;  // the item order is no longer needed below
        idx.resize(n);
        for (size_t k = 0; k < n; ++k) idx[k] = (int)k;
        std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost[a] > cost[b]; });
        for (size_t r = 0; r < n; ++r) dealt[dealt_position((long long)r, nq, q_begin)] = refs[idx[r]];
    }
    out.n_tasks = (int)n;
    out.nq = nq;
    out.n_slots = n_slots;
    out.interactions = inter;
    return PGH_OK;
}

void write_tasks(const HostPlan &hp, Task *dst)
{
    const std::vector<PlanChunk> &chunks = hp.chunks;
    for (size_t k = 0; k < hp.dealt.size(); ++k) {
        const PlanRef &r = hp.dealt[k];
        const PlanWork &wk = hp.work[r.work];
        const PlanChunk &a = chunks[wk.a];
        const bool pair = wk.b >= 0;
        static const PlanChunk kNone{0, 0, 0, 0, 1};
        const PlanChunk &b = pair ? chunks[wk.b] : kNone;
        dst[k] = work_task(a.i_off, a.n_i, a.j_off, a.n_j, pair, b.i_off, b.n_i, b.j_off, b.n_j,
                           WorkCut{wk.parts, wk.per, 0}, r.part, wk.slot);
    }
}

int plan_descs(const pgh_item *items, int n_items, int ni_total, int nj_total, int waves,
               DescPlan &out, std::string &err)
{
    Scratch &S = scratch();
    std::vector<int> &order = S.order;
    long long inter = 0;
    {
        const int st = validate_items(items, n_items, ni_total, nj_total, order, out.ordered,
                                      &inter, err);
        if (st) return st;
    }
    // the same chunks as plan_tasks, which must be of 64 here
    waves = std::max(1, waves);
    long long n64 = 0, total = 0;
    for (int t : order) {
        const pgh_item &it = items[t];
        const int n_full = it.n_i >> 6, n_last = it.n_i & 63;
        n64 += n_full + (n_last ? 1 : 0);
        total += n_full * std::max(1LL, (long long)it.n_j);
        if (n_last) total += std::max(1LL, lane_steps(it.n_j, chunk_js(n_last)));
    }
    if (n64 < waves) return kPlanOnHost;
    const long long part_iters = part_length(total, waves);
    // every cost is at most part_iters + 64 (a part of at most part_iters
    // steps rounded up to whole tiles), so kmax - cost fits the sort keys
    const long long kmax = part_iters + 64;
    if (kmax >= (1LL << 31)) return kPlanOnHost;
    // the partly filled chunk of each item is its last; those with a list
    // are the pairing candidates, by item (the chunk order)
    std::vector<int> &cand = S.cand;
    cand.clear();
    for (size_t k = 0; k < order.size(); ++k) {
        const pgh_item &it = items[order[k]];
        if ((it.n_i & 63) && it.n_j > 0) cand.push_back((int)k);
    }
    pair_chunks(S, cand, [&](int k) { return items[order[k]].n_i & 63; },
                [&](int k) { return items[order[k]].n_j; }, S.pairs);
    std::vector<char> &taken = S.taken;
    taken.assign(order.size(), 0);
    std::vector<PlanDesc> &desc = out.desc;
    desc.clear();
    long long n_tasks = 0, n_slots = 0, n_split = 0;
    auto add = [&](PlanDesc d) {
        int tasks = 0, slots = 0, splits = 0;
        desc_counts(d, part_iters, &tasks, &slots, &splits);
        d.task0 = (int)n_tasks;
        d.slot0 = (int)n_slots;
        d.split0 = (int)n_split;
        n_tasks += tasks;
        n_slots += slots;
        n_split += splits;
        desc.push_back(d);
    };
    for (const auto &pr : S.pairs) {
        const pgh_item &a = items[order[pr.first]], &b = items[order[pr.second]];
        const int na = a.n_i & 63, nb = b.n_i & 63;
        taken[pr.first] = taken[pr.second] = 1;
        add({a.i_off + a.n_i - na, na, a.j_off, a.n_j, b.i_off + b.n_i - nb, nb, b.j_off, b.n_j,
             0, 0, 0, 0});
    }
    for (size_t k = 0; k < order.size(); ++k) {
        const pgh_item &it = items[order[k]];
        const int n = taken[k] ? it.n_i - (it.n_i & 63) : it.n_i;
        if (n > 0) add({it.i_off, n, it.j_off, it.n_j, 0, 0, 0, 0, 0, 0, 0, 0});
        if (n_tasks > (1LL << 30) || n_slots > (1LL << 30))
            return fail_msg(err, PGH_ERANGE, "the plan exceeds 2^30 tasks");
    }
    out.n_tasks = (int)n_tasks;
    out.n_slots = (int)n_slots;
    out.n_split = (int)n_split;
    out.nq = deal_layout((size_t)n_tasks, out.q_begin);
    out.part_iters = part_iters;
    out.kmax = (unsigned)kmax;
    out.interactions = inter;
    return PGH_OK;
}

void plan_adjoint_tasks(const std::vector<pgh_item> &ordered, int waves, std::vector<Task> &out_j,
                        std::vector<Task> &out_i)
{
    const std::vector<pgh_item> &ord = ordered;
    waves = std::max(1, waves);
    // j-major tasks of the table adjoint: chunks of <= 64 j-entries of a
    // list against its i-group (chunks of 32 or 16, 2 or 4 lanes per entry,
    // when chunks of 64 would fill less than half of the resident waves)
    int jc = 64;
    long long n_j = 0;
    for (;;) {
        n_j = 0;
        for (const pgh_item &it : ord) n_j += (it.n_j + jc - 1) / jc;
        if (2 * n_j >= waves || jc == 16) break;
        jc /= 2;
    }
    // i-major tasks (the i-side position gradient, its own list independent
    // of the forward's chunking): i-chunks of <= 64 against j-ranges of
    // <= 512, added with atomics, so no partial sums; chunks of 32 or 16 (2
    // or 4 lanes per i-particle) while the two kinds together would fill
    // less than the resident waves twice over
    int ic = 64;
    for (;;) {
        long long n_i = 0;
        for (const pgh_item &it : ord)
            n_i += (long long)((it.n_i + ic - 1) / ic) * ((it.n_j + 511) / 512);
        if (n_i + n_j >= 2LL * waves || ic == 16) break;
        ic /= 2;
    }
    std::vector<Task> &it_tasks = out_i;
    it_tasks.clear();
    for (const pgh_item &it : ord) {
        for (int s0 = 0; s0 < it.n_i; s0 += ic)
            for (int q0 = 0; q0 < it.n_j; q0 += 512)
                it_tasks.push_back({it.i_off + s0, std::min(ic, it.n_i - s0), it.j_off + q0,
                                    std::min(512, it.n_j - q0), 0, 1, 0, 0, 0, 0, 0, 0});
    }
    // longest first, a task's length in lane steps (n_j over the lanes per
    // i-particle)
    std::stable_sort(it_tasks.begin(), it_tasks.end(), [](const Task &a, const Task &b) {
        return lane_steps(a.n_j, chunk_js(a.n_i)) > lane_steps(b.n_j, chunk_js(b.n_i));
    });
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
