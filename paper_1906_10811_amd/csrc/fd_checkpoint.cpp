// fd_checkpoint.cpp -- binomial (revolve-style) checkpoint schedules for the
// reverse sweep of fd_gradient.
//
// To reverse nt time steps the adjoint needs, for n = nt-1 down to 0, the
// state (u^n, u^{n-1}) from which one forward step gives u^{n+1} and the
// imaging bracket of level n.  With `slots` snapshot slots besides the
// initial state, the schedule minimising the number of forward steps is
// built by dynamic programming over the split point of each segment:
//
//   T(l, c) = 0                                   l = 1
//   T(l, 0) = l (l - 1) / 2                       advance from the segment start each time
//   T(l, c) = min_{1 <= m < l} m + T(l - m, c - 1) + T(m, c)
//
// i.e. advance m steps, store a snapshot, reverse the last l - m steps with
// one slot fewer, then reverse the first m steps from the segment start with
// the slot returned.  This is the optimal offline schedule whose cost the
// binomial checkpointing theorem of Griewank and Walther gives in closed
// form; the DP finds the split points directly instead of using their
// placement rules.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "../../include/fd.h"
#include "fd_api_internal.h"

namespace {

struct Plan {
    int nt, slots;
    std::vector<long long> T;   // (nt+1) x (slots+1), forward steps
    std::vector<int> M;         // argmin split
    long long &t(int l, int c) { return T[(size_t)l * (slots + 1) + c]; }
    int &m(int l, int c) { return M[(size_t)l * (slots + 1) + c]; }
};

void solve(Plan &p) {
    p.T.assign((size_t)(p.nt + 1) * (p.slots + 1), 0);
    p.M.assign((size_t)(p.nt + 1) * (p.slots + 1), 0);
    for (int l = 1; l <= p.nt; ++l) {
        p.t(l, 0) = (long long)l * (l - 1) / 2;
        for (int c = 1; c <= p.slots; ++c) {
            if (l == 1) {
                p.t(l, c) = 0;
                continue;
            }
            long long best = LLONG_MAX;
            int arg = 1;
            for (int mm = 1; mm < l; ++mm) {
                const long long v = mm + p.t(l - mm, c - 1) + p.t(mm, c);
                if (v < best) {
                    best = v;
                    arg = mm;
                }
            }
            p.t(l, c) = best;
            p.m(l, c) = arg;
        }
    }
}

struct Emitter {
    fd_ckpt_action *out;
    int cap;
    int n = 0;
    int horizon = 0;   // steps computed so far for the first time: [0, horizon)
    bool overflow = false;
    void push(int kind, int step, int count, int slot) {
        if (n < cap && out) {
            fd_ckpt_action &a = out[n];
            a.kind = kind;
            a.step = step;
            a.count = count;
            a.slot = slot;
            a.first = 0;
            if (kind == FD_ACT_ADVANCE || kind == FD_ACT_YOUTURN) {
                const int end = step + (kind == FD_ACT_ADVANCE ? count : 1);
                a.first = end > horizon ? 1 : 0;
                if (end > horizon) horizon = end;
            }
        } else if (out) {
            overflow = true;
        }
        ++n;
    }
};

// Reverse steps [s, s + l) with the state of level s in slot `at` and
// free slots `c`, whose indices are next_free .. next_free + c - 1.
void emit(Plan &p, Emitter &e, int s, int l, int c, int at, int next_free) {
    if (l == 1) {
        e.push(FD_ACT_RESTORE, s, 0, at);
        e.push(FD_ACT_YOUTURN, s, 1, -1);
        return;
    }
    if (c == 0) {
        for (int k = l - 1; k >= 0; --k) {
            e.push(FD_ACT_RESTORE, s, 0, at);
            if (k > 0) e.push(FD_ACT_ADVANCE, s, k, -1);
            e.push(FD_ACT_YOUTURN, s + k, 1, -1);
        }
        return;
    }
    const int mm = p.m(l, c);
    e.push(FD_ACT_RESTORE, s, 0, at);
    e.push(FD_ACT_ADVANCE, s, mm, -1);
    e.push(FD_ACT_STORE, s + mm, 0, next_free);
    emit(p, e, s + mm, l - mm, c - 1, next_free, next_free + 1);
    emit(p, e, s, mm, c, at, next_free);
}

}  // namespace

int fdi_checkpoint_plan(int nt, int slots, std::vector<fd_ckpt_action> *actions, long long *fwd) {
    if (nt < 1 || slots < 0) return fdi_fail(FD_ERR_ARG, "nt >= 1 and slots >= 0");
    if ((long long)nt * nt * (slots + 1) > 4000000000LL)
        return fdi_fail(FD_ERR_ARG, "schedule too large (nt %d, slots %d)", nt, slots);
    Plan p{nt, std::min(slots, nt)};
    solve(p);
    Emitter cnt{nullptr, 0};
    emit(p, cnt, 0, nt, p.slots, 0, 1);
    actions->resize(cnt.n);
    Emitter e{actions->data(), cnt.n};
    emit(p, e, 0, nt, p.slots, 0, 1);
    if (fwd) *fwd = p.t(nt, p.slots);
    return FD_OK;
}

extern "C" int fd_checkpoint_schedule(int nt, int slots, fd_ckpt_action *actions, int capacity,
                                      int *n_actions, long long *forward_steps) {
    try {
        if (!n_actions) return fdi_fail(FD_ERR_ARG, "null n_actions");
        std::vector<fd_ckpt_action> v;
        int rc = fdi_checkpoint_plan(nt, slots, &v, forward_steps);
        if (rc) return rc;
        *n_actions = (int)v.size();
        if (actions) {
            if (capacity < (int)v.size()) return fdi_fail(FD_ERR_NOMEM, "capacity %d < %zu actions", capacity, v.size());
            std::copy(v.begin(), v.end(), actions);
        }
        return FD_OK;
    } catch (...) {
        return fdi_fail(FD_ERR_NOMEM, "host allocation failed");
    }
}
