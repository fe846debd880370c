// Scheduling of one server pass: which (request, database position) pairs the
// pass serves.  Pure host logic (no HIP), used by the server in sw_host.cpp
// and tested on its own.
//
// The database is cut into positions (chunks of lane-per-subject groups, and
// the long list).  Each request keeps its own next position and the number it
// still has to visit; it is done when that number reaches 0.  A pass:
//  * first advances the oldest request (lowest ticket) by one position, so no
//    request starves whatever arrives after it;
//  * then lets the requests with the least work left (cells of their remaining
//    positions) take their next positions, as many as the budget allows, so a
//    short query can finish in one pass instead of riding every pass of a long
//    one (shortest remaining work first, batched);
//  * is full once it holds `pass_cells * scale` cells and `pass_items`
//    lane-per-subject items (enough per resident workgroup to keep the work
//    queue's tail small); scale = active requests / 4, from 1 up to 16, so that
//    under load a pass's fixed costs stay small against its work;
//  * never holds more (request, subject) pairs than `pair_cap` (the capacity
//    of the overflow list), except that the first position is always taken.
#pragma once

#include <algorithm>
#include <cstdint>
#include <utility>
#include <vector>

namespace swmi {

struct SchedReq {
    uint64_t ticket = 0;     // arrival order
    int64_t qlen = 0;
    int32_t next = 0;        // next position to visit
    int32_t remaining = 0;   // positions still to visit
};

struct SchedPos {
    int64_t res = 0;         // subject residues at this position
    int64_t items = 0;       // lane-per-subject work items per request
    int64_t subj = 0;        // subjects (pairs per request)
};

struct SchedBudget {
    int64_t pass_cells = 1;
    int64_t pass_items = 0;
    int64_t pair_cap = 0;
};

struct SchedTake {
    int32_t req;             // index into the request vector
    int32_t pos;
};

// Cells of the positions request r still has to visit.
inline int64_t sched_left_cells(const SchedReq &r, const std::vector<SchedPos> &pos) {
    const int32_t n_pos = (int32_t)pos.size();
    int64_t c = 0;
    for (int32_t x = 0, p = r.next; x < r.remaining; ++x, p = (p + 1) % n_pos) c += pos[p].res;
    return c * r.qlen;
}

// Appends this pass's work to `out` (in the order taken) and advances `next`
// and `remaining` of every request taken.
inline void sched_plan_pass(std::vector<SchedReq> &reqs, const std::vector<SchedPos> &pos,
                            const SchedBudget &b, std::vector<SchedTake> &out) {
    const int32_t n_pos = (int32_t)pos.size();
    std::vector<int32_t> act;
    for (int32_t i = 0; i < (int32_t)reqs.size(); ++i)
        if (reqs[i].remaining > 0) act.push_back(i);
    if (act.empty() || n_pos == 0) return;
    std::vector<std::pair<int64_t, int32_t>> order;
    for (int32_t i : act) order.push_back({sched_left_cells(reqs[i], pos), i});
    std::stable_sort(order.begin(), order.end(), [&](const auto &x, const auto &y) {
        return x.first != y.first ? x.first < y.first : reqs[x.second].ticket < reqs[y.second].ticket;
    });
    int32_t oldest = act[0];
    for (int32_t i : act)
        if (reqs[i].ticket < reqs[oldest].ticket) oldest = i;
    const size_t first = out.size();
    int64_t cells = 0, items = 0, pairs = 0;
    auto take = [&](int32_t i) -> bool {
        SchedReq &r = reqs[i];
        if (r.remaining == 0) return false;
        const int32_t p = r.next;
        if (out.size() > first && pairs + pos[p].subj > b.pair_cap) return false;
        out.push_back({i, p});
        cells += pos[p].res * r.qlen;
        items += pos[p].items;
        pairs += pos[p].subj;
        r.next = (p + 1) % n_pos;
        r.remaining--;
        return true;
    };
    const int64_t scale = std::min<int64_t>(16, std::max<int64_t>(1, (int64_t)act.size() / 4));
    auto full = [&] { return cells >= b.pass_cells * scale && items >= b.pass_items; };
    take(oldest);
    for (const auto &o : order) {
        if (full()) break;
        while (!full() && take(o.second)) {
        }
    }
}

}  // namespace swmi
