// Binomial checkpointing for reversing l explicit steps with c snapshot slots
// (Griewank's binomial checkpointing, as in the Revolve schedule of Griewank
// and Walther): with the repetition number r, the smallest r with
// beta(c, r) = C(c + r, c) >= l, no step is recomputed more than r times and
// the number of forward steps is r l - beta(c + 1, r - 1), the minimum over all
// schedules that hold at most c states at a time.
//
// Recursion: to reverse steps [a, b) with c slots, state a in one of them,
// advance to a split point m, store state m, reverse [m, b) with the c - 1
// slots left, release the slot of m, and reverse [a, m) with c slots.  The cost
// is minimal when the right part fits repetition r on c - 1 slots and the left
// part repetition r - 1 on c slots (Pascal's rule beta(c, r) = beta(c, r - 1) +
// beta(c - 1, r) splits the reachable range exactly):
//   beta(c, r - 2) <= m - a <= beta(c, r - 1),
//   beta(c - 1, r - 1) <= b - m <= beta(c - 1, r).
// Host code only; the executor lives in the C ABI.
#include <algorithm>
#include <vector>

#include "pbf_internal.h"

namespace pbf {
namespace {

constexpr long long kSat = 1LL << 62;

// beta(c, r) = C(c + r, c), saturated at 2^62; zero for r < 0
long long beta(int c, int r)
{
    if (r < 0 || c < 0) return 0;
    const int k = std::min(c, r);
    const long long n = (long long)c + r;
    __int128 v = 1;
    for (int i = 1; i <= k; ++i) {
        v = v * (n - k + i) / i;  // C(n - k + i, i), exact
        if (v >= kSat) return kSat;
    }
    return (long long)v;
}

int repetitions(long long l, int c)
{
    int r = 0;
    while (beta(c, r) < l) ++r;
    return r;
}

struct Item {
    bool release;  // true: give slot back
    int a, b, c, slot;
};

}  // namespace

long long revolve_min_advances(long long l, int c)
{
    const int r = repetitions(l, c);
    if (r == 0) return 0;
    const long long b = beta(c + 1, r - 1);
    return r * l - b;
}

bool revolve_schedule(int l, int c, std::vector<pbf_revolve_action> &acts, long long *advances)
{
    acts.clear();
    if (l < 1 || c < 1) return false;
    c = std::min(c, l);  // more slots than steps are never used
    int cur = 0;
    long long adv = 0;
    auto emit = [&](int kind, int step, int slot) { acts.push_back(pbf_revolve_action{kind, step, slot}); };
    auto restore = [&](int a, int slot) {
        if (cur != a) {
            emit(PBF_ACT_RESTORE, a, slot);
            cur = a;
        }
    };
    auto advance = [&](int to) {
        if (to > cur) {
            emit(PBF_ACT_ADVANCE, to, -1);
            adv += to - cur;
            cur = to;
        }
    };
    std::vector<int> free_slots;
    for (int k = c - 1; k >= 1; --k) free_slots.push_back(k);
    emit(PBF_ACT_STORE, 0, 0);
    std::vector<Item> stack{{false, 0, l, c, 0}};
    while (!stack.empty()) {
        const Item it = stack.back();
        stack.pop_back();
        if (it.release) {
            free_slots.push_back(it.slot);
            continue;
        }
        const int a = it.a, b = it.b, cc = it.c, sa = it.slot;
        const long long len = (long long)b - a;
        if (len == 1) {
            restore(a, sa);
            emit(PBF_ACT_TURN, a, -1);
            continue;
        }
        if (cc == 1 || free_slots.empty()) {
            for (int i = b - 1; i >= a; --i) {
                restore(a, sa);
                advance(i);
                emit(PBF_ACT_TURN, i, -1);
            }
            continue;
        }
        const int r = repetitions(len, cc);
        long long m = std::max(beta(cc, r - 2), len - beta(cc - 1, r));
        m = std::min(std::max(m, 1LL), len - 1);
        restore(a, sa);
        advance(a + (int)m);
        const int s2 = free_slots.back();
        free_slots.pop_back();
        emit(PBF_ACT_STORE, a + (int)m, s2);
        stack.push_back({false, a, a + (int)m, cc, sa});
        stack.push_back({true, 0, 0, 0, s2});
        stack.push_back({false, a + (int)m, b, cc - 1, s2});
    }
    if (advances) *advances = adv;
    return true;
}

}  // namespace pbf
