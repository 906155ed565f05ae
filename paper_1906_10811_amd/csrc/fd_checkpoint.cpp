// fd_checkpoint.cpp -- binomial (revolve-style) checkpoint schedules for the
// reverse sweep of fd_gradient.
//
// To reverse nt time steps the adjoint needs, for n = nt-1 down to 0, the
// state (u^n, u^{n-1}) from which one forward step gives u^{n+1} and the
// imaging bracket of level n.  With c snapshot slots besides the initial
// state, the fewest forward steps T(l, c) to reverse l steps satisfy
//
//   T(1, c) = 0,   T(l, 0) = l (l - 1) / 2,
//   T(l, c) = min_{1 <= m < l} m + T(l - m, c - 1) + T(m, c)
//
// (advance m steps, store a snapshot, reverse the last l - m steps with one
// slot fewer, then the first m steps with the slot returned).  The binomial
// checkpointing theorem of Griewank and Walther gives the minimum in closed
// form: with s = c + 1 checkpoints (the initial state included) and r the
// least integer with C(s + r, s) >= l,
//
//   T(l, c) = r l - C(s + r, s + 1),
//
// so T(l + 1, c) - T(l, c) = r(l + 1): T is convex in l, and so is the cost
// of a split as a function of m.  The schedule takes the smallest optimal m
// of each split, found by bisection on the sign of the cost's difference
//
//   D(m) = 1 + r_{s}(m + 1) - r_{s-1}(l - m),
//
// O(log l) evaluations of r per split instead of a table of all (l, c).
#include <algorithm>
#include <climits>
#include <cstdint>
#include <vector>

#include "../../include/fd.h"
#include "fd_api_internal.h"

namespace {

// r_s(n): the least r >= 0 with C(s + r, s) >= n (s >= 1, n >= 1)
long long reps(long long n, int s) {
    if (n <= 1) return 0;
    if (s == 1) return n - 1;   // C(1 + r, 1) = r + 1
    long long b = 1, r = 0;     // b = C(s + r, r)
    while (b < n) {
        b = b * (s + r + 1) / (r + 1);   // exact: C(s + r + 1, r + 1)
        ++r;
    }
    return r;
}

// T(l, c) in closed form
long long fwd_steps(long long l, int c) {
    if (l <= 1) return 0;
    if (c == 0) return l * (l - 1) / 2;
    const int s = c + 1;
    const long long r = reps(l, s);
    long long b = 1;   // C(s + r, s + 1) = C(s + r, r - 1)
    for (long long k = 0; k < r - 1; ++k) b = b * (s + 2 + k) / (k + 1);
    return r * l - (r >= 1 ? b : 0);
}

// smallest optimal split of (l, c), c >= 1, l >= 2
int split(int l, int c) {
    auto d = [&](int m) { return 1 + reps(m + 1, c + 1) - reps(l - m, c); };
    int lo = 1, hi = l - 1;   // the answer is the first m in [1, l - 2] with D(m) >= 0, else l - 1
    while (lo < hi) {
        const int mid = lo + (hi - lo) / 2;
        if (d(mid) >= 0) hi = mid;
        else lo = mid + 1;
    }
    return lo;
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
void emit(Emitter &e, int s, int l, int c, int at, int next_free) {
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
    const int mm = split(l, c);
    e.push(FD_ACT_RESTORE, s, 0, at);
    e.push(FD_ACT_ADVANCE, s, mm, -1);
    e.push(FD_ACT_STORE, s + mm, 0, next_free);
    emit(e, s + mm, l - mm, c - 1, next_free, next_free + 1);
    emit(e, s, mm, c, at, next_free);
}

}  // namespace

int fdi_checkpoint_plan(int nt, int slots, std::vector<fd_ckpt_action> *actions, long long *fwd) {
    if (nt < 1 || slots < 0) return fdi_fail(FD_ERR_ARG, "nt >= 1 and slots >= 0");
    // at most about four actions per time step (restore, advance, store,
    // reverse), counted in an int
    if (nt > INT_MAX / 8) return fdi_fail(FD_ERR_ARG, "schedule too large (nt %d)", nt);
    const int c = std::min(slots, nt);
    const long long total = fwd_steps(nt, c);
    Emitter cnt{nullptr, 0};
    emit(cnt, 0, nt, c, 0, 1);
    actions->resize(cnt.n);
    Emitter e{actions->data(), cnt.n};
    emit(e, 0, nt, c, 0, 1);
    if (fwd) *fwd = total;
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
