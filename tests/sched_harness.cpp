// Drives the server's pass scheduler (sw_sched.h) on a scripted scenario.
// stdin:  n_pos pass_cells pass_items pair_cap
//         n_pos lines: res items subj
//         n_req
//         n_req lines: qlen arrival_pass        (ticket = line order)
// stdout: "pass <p> <ticket>:<pos> ..." per pass, then "done <ticket> <pass>" per request.
#include <cstdio>
#include <vector>

#include "sw_sched.h"

int main() {
    int n_pos = 0;
    long long pc = 0, pi = 0, cap = 0;
    if (scanf("%d %lld %lld %lld", &n_pos, &pc, &pi, &cap) != 4) return 2;
    std::vector<swmi::SchedPos> pos(n_pos);
    for (auto &p : pos)
        if (scanf("%lld %lld %lld", (long long *)&p.res, (long long *)&p.items, (long long *)&p.subj) != 3) return 2;
    int n_req = 0;
    if (scanf("%d", &n_req) != 1) return 2;
    std::vector<long long> qlen(n_req), arrive(n_req);
    for (int i = 0; i < n_req; ++i)
        if (scanf("%lld %lld", &qlen[i], &arrive[i]) != 2) return 2;
    const swmi::SchedBudget b{pc, pi, cap};
    std::vector<swmi::SchedReq> active;
    std::vector<int> ticket_of;   // active index -> ticket
    std::vector<int> done(n_req, -1);
    int finished = 0;
    for (int pass = 0; finished < n_req && pass < 100000; ++pass) {
        for (int i = 0; i < n_req; ++i)
            if (arrive[i] == pass) {
                active.push_back(swmi::SchedReq{(unsigned long long)i, qlen[i], 0, n_pos});
                ticket_of.push_back(i);
            }
        std::vector<swmi::SchedTake> takes;
        swmi::sched_plan_pass(active, pos, b, takes);
        printf("pass %d", pass);
        for (const auto &t : takes) printf(" %d:%d", ticket_of[t.req], t.pos);
        printf("\n");
        for (size_t i = 0; i < active.size();) {
            if (active[i].remaining == 0) {
                done[ticket_of[i]] = pass;
                ++finished;
                active.erase(active.begin() + i);
                ticket_of.erase(ticket_of.begin() + i);
            } else {
                ++i;
            }
        }
    }
    for (int i = 0; i < n_req; ++i) printf("done %d %d\n", i, done[i]);
    return 0;
}
