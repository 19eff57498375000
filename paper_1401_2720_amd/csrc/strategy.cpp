// Parallel pivot strategies (Section 3).
//
// A p-strategy of even order N has N-1 parallel steps (p-steps) of N/2
// disjoint pivot pairs and visits every pair once per sweep, eq. (3.1).
// The strategy closest to a sequential order O (Definition 3.1) is the one
// whose pairs, read step by step, have the lexicographically smallest
// sequence of positions in O.  Algorithm 3.1 builds it by taking the
// lexicographically first set of N/2 disjoint unused pairs that still lets
// the remaining pairs be completed, backtracking otherwise.  The round-robin
// ordering, one of the strategies Section 6 compares against, is built
// directly.  It is only
// affordable for small orders, so (following Section 3) a table of order
// 2^k * o is built from order 2o by k-1 expansions of Algorithm 3.2, which
// turns every p-step of order N into two p-steps of order 2N.  The reverse
// strategies list the pairs in the opposite order.
#include "jsvd_internal.h"

#include <algorithm>
#include <map>
#include <mutex>

namespace jsvd {

namespace {

// Sequential cyclic orders as lists of zero-based pairs.
std::vector<Pair> sequential(int n, bool row_cyclic) {
    std::vector<Pair> v;
    v.reserve(static_cast<size_t>(n) * (n - 1) / 2);
    if (row_cyclic) {
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) v.push_back({i, j});
    } else {
        for (int j = 1; j < n; ++j)
            for (int i = 0; i < j; ++i) v.push_back({i, j});
    }
    return v;
}

// Algorithm 3.1 by depth-first search over positions in the sequential
// order.  'used' marks pairs already placed in earlier p-steps.
class ClosestSearch {
  public:
    ClosestSearch(int n, bool row) : n_(n), half_(n / 2), seq_(sequential(n, row)), used_(seq_.size(), 0) {}

    bool run(Table &out) {
        steps_.clear();
        if (!level(static_cast<int>(seq_.size()))) return false;
        out.clear();
        for (const auto &st : steps_) {
            Step s;
            for (int pos : st) s.push_back(seq_[pos]);
            out.push_back(s);
        }
        return true;
    }

  private:
    // One recursion level of Algorithm 3.1: enumerate candidate p-steps in
    // lexicographic order of positions and recurse on the rest.
    bool level(int remaining) {
        if (remaining == 0) return true;
        std::vector<int> chosen;
        std::vector<char> covered(n_, 0);
        return enumerate(0, chosen, covered, remaining);
    }

    // Every index not yet covered must still be reachable by an unused pair
    // at a position >= start whose other index is also uncovered.
    bool feasible(int start, const std::vector<char> &covered) const {
        std::vector<char> reach(n_, 0);
        for (size_t k = start; k < seq_.size(); ++k) {
            if (used_[k]) continue;
            const Pair &pr = seq_[k];
            if (!covered[pr.first] && !covered[pr.second]) reach[pr.first] = reach[pr.second] = 1;
        }
        for (int i = 0; i < n_; ++i)
            if (!covered[i] && !reach[i]) return false;
        return true;
    }

    bool enumerate(int start, std::vector<int> &chosen, std::vector<char> &covered, int remaining) {
        if (static_cast<int>(chosen.size()) == half_) {
            for (int pos : chosen) used_[pos] = 1;
            steps_.push_back(chosen);
            if (level(remaining - half_)) return true;
            steps_.pop_back();
            for (int pos : chosen) used_[pos] = 0;
            return false;  // try the next candidate (backtrack)
        }
        if (!feasible(start, covered)) return false;
        for (size_t k = start; k < seq_.size(); ++k) {
            if (used_[k]) continue;
            const Pair &pr = seq_[k];
            if (covered[pr.first] || covered[pr.second]) continue;
            covered[pr.first] = covered[pr.second] = 1;
            chosen.push_back(static_cast<int>(k));
            if (enumerate(static_cast<int>(k) + 1, chosen, covered, remaining)) return true;
            chosen.pop_back();
            covered[pr.first] = covered[pr.second] = 0;
        }
        return false;
    }

    int n_, half_;
    std::vector<Pair> seq_;
    std::vector<char> used_;
    std::vector<std::vector<int>> steps_;
};

// Algorithm 3.2: order N -> order 2N.  The first p-step pairs (2k, 2k+1)
// (zero-based); p-step i >= 1 of the result comes from p-step (i+1)/2 - 1
// of the input: even one-based i gives the NW and SE pairs of each 2x2
// block, odd i the NE and SW pairs (SW first for the column-cyclic family).
Table expand(const Table &in, bool row_cyclic) {
    const int n = static_cast<int>(in.size()) + 1;
    Table out;
    Step first;
    for (int k = 0; k < n; ++k) first.push_back({2 * k, 2 * k + 1});
    out.push_back(first);
    for (int i = 2; i <= 2 * n - 1; ++i) {  // one-based step index
        const Step &src = in[i / 2 - 1];
        Step s;
        for (const Pair &pq : src) {
            const int p = pq.first, q = pq.second;
            if (i % 2 == 0) {
                s.push_back({2 * p, 2 * q});
                s.push_back({2 * p + 1, 2 * q + 1});
            } else if (row_cyclic) {
                s.push_back({2 * p, 2 * q + 1});
                s.push_back({2 * p + 1, 2 * q});
            } else {
                s.push_back({2 * p + 1, 2 * q});
                s.push_back({2 * p, 2 * q + 1});
            }
        }
        out.push_back(s);
    }
    return out;
}

// Round-robin ordering of order N in Brent and Luk's layout: two rows of
// N/2 places, pair k of a p-step joins top[k] and bot[k]; the first step
// pairs (0,1), (2,3), ...; between steps top[0] stays and every other index
// moves one place round the ring top[1] -> top[2] -> ... -> top[N/2-1] ->
// bot[N/2-1] -> ... -> bot[0] -> top[1].  After N - 1 steps every pair has
// met once.
Table round_robin(int order) {
    const int h = order / 2;
    std::vector<int> top(h), bot(h);
    for (int k = 0; k < h; ++k) {
        top[k] = 2 * k;
        bot[k] = 2 * k + 1;
    }
    Table t;
    for (int s = 0; s + 1 < order; ++s) {
        Step st;
        for (int k = 0; k < h; ++k) st.push_back({std::min(top[k], bot[k]), std::max(top[k], bot[k])});
        t.push_back(st);
        if (h > 1) {
            std::vector<int> nt(h), nb(h);
            nt[0] = top[0];
            nt[1] = bot[0];
            for (int k = 2; k < h; ++k) nt[k] = top[k - 1];
            for (int k = 0; k + 1 < h; ++k) nb[k] = bot[k + 1];
            nb[h - 1] = top[h - 1];
            top.swap(nt);
            bot.swap(nb);
        }
    }
    return t;
}

bool split_order(int order, int &k, int &o) {
    if (order < 2 || order % 2) return false;
    k = 0;
    o = order;
    while (o % 2 == 0) {
        o /= 2;
        ++k;
    }
    return o == 1 || o == 3 || o == 5 || o == 7 || o == 9 || o == 11;
}

}  // namespace

int strategy_order(int nb) {
    int n = nb < 2 ? 2 : nb;
    if (n % 2) ++n;
    int k, o;
    while (!split_order(n, k, o)) n += 2;
    return n;
}

bool make_table(int order, int kind, Table &out) {
    static std::mutex mu;
    static std::map<std::pair<int, int>, Table> cache;
    int k, o;
    if (!split_order(order, k, o) || order > 4096) return false;
    if (kind < JSVD_STRAT_RREV || kind > JSVD_STRAT_RR) return false;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find({order, kind});
    if (it != cache.end()) {
        out = it->second;
        return true;
    }
    if (kind == JSVD_STRAT_RR) {
        cache[{order, kind}] = round_robin(order);
        out = cache[{order, kind}];
        return true;
    }
    const bool row = (kind == JSVD_STRAT_R || kind == JSVD_STRAT_RREV);
    const bool rev = (kind == JSVD_STRAT_RREV || kind == JSVD_STRAT_CREV);
    Table t;
    int cur;
    if (o == 1) {
        t = {Step{{0, 1}}};
        cur = 2;
    } else {
        ClosestSearch s(2 * o, row);
        if (!s.run(t)) return false;
        cur = 2 * o;
    }
    while (cur < order) {
        t = expand(t, row);
        cur *= 2;
    }
    if (rev) {
        Table r(t.rbegin(), t.rend());
        for (auto &st : r) std::reverse(st.begin(), st.end());
        t.swap(r);
    }
    cache[{order, kind}] = t;
    out = t;
    return true;
}

// The pairs of one parallel step are disjoint, so the slot a pair takes in
// the inner kernels does not change any result.  There, slot s is lanes
// 8s .. 8s + 7, lane x reading rows x + 8r of the pair's columns p and q
// (column-major, leading dimension = 1 mod 32 doubles), so that its 8 lanes
// hit 8 consecutive 8-byte banks starting at p mod 16 (32 four-byte banks,
// read in 16-lane halves) or p mod 32 (64 banks, 32-lane halves).  Two slots
// 2k, 2k + 1 are conflict-free under the first model when their p differ by
// 8 mod 16 and their q too; four slots 4k .. 4k + 3 under the second when
// their p mod 32 are c, c + 8, c + 16, c + 24 in that order, and their q mod
// 32 likewise (within such a quadruple the slots are ordered so that its two
// couples satisfy the first model too where they can).  Each step is
// reordered greedily: such quadruples first, then such couples, then the
// rest.
void order_for_banks(Table &t) {
    for (Step &st : t) {
        const int np = (int)st.size();
        std::vector<char> used(np, 0);
        Step out;
        out.reserve(np);
        auto qpos = [](int v) { return (v % 32) / 8; };
        // quadruples: the same p mod 8 and q mod 8, p mod 32 and q mod 32 in
        // the four eighths of 32 (each once), slot order by p's eighth
        for (int a = 0; a < np && np % 4 == 0; ++a) {
            if (used[a]) continue;
            int pick[4] = {-1, -1, -1, -1};
            pick[qpos(st[a].first)] = a;
            int qmask = 1 << qpos(st[a].second);
            for (int b = 0; b < np; ++b) {
                if (used[b] || b == a) continue;
                if (st[b].first % 8 != st[a].first % 8 || st[b].second % 8 != st[a].second % 8)
                    continue;
                const int pp = qpos(st[b].first), qq = qpos(st[b].second);
                if (pick[pp] >= 0 || (qmask >> qq & 1)) continue;
                pick[pp] = b;
                qmask |= 1 << qq;
            }
            if (pick[0] >= 0 && pick[1] >= 0 && pick[2] >= 0 && pick[3] >= 0) {
                // an order whose two couples are also conflict-free in 16-lane
                // halves (p and q each an odd number of eighths apart), if any
                int ord[4] = {pick[0], pick[1], pick[2], pick[3]};
                int perm[4] = {0, 1, 2, 3};
                do {
                    auto odd = [&](int u, int v) {
                        const Pair &x = st[pick[perm[u]]], &y = st[pick[perm[v]]];
                        return ((qpos(x.first) - qpos(y.first)) & 1) && ((qpos(x.second) - qpos(y.second)) & 1);
                    };
                    if (odd(0, 1) && odd(2, 3)) {
                        for (int k = 0; k < 4; ++k) ord[k] = pick[perm[k]];
                        break;
                    }
                } while (std::next_permutation(perm, perm + 4));
                for (int k = 0; k < 4; ++k) {
                    used[ord[k]] = 1;
                    out.push_back(st[ord[k]]);
                }
            }
        }
        // couples: p and q both 8 apart mod 16
        for (int a = 0; a < np; ++a) {
            if (used[a]) continue;
            for (int b = a + 1; b < np; ++b) {
                if (used[b]) continue;
                if ((st[a].first - st[b].first + 16) % 16 == 8 &&
                    (st[a].second - st[b].second + 16) % 16 == 8) {
                    used[a] = used[b] = 1;
                    out.push_back(st[a]);
                    out.push_back(st[b]);
                    break;
                }
            }
        }
        for (int a = 0; a < np; ++a)
            if (!used[a]) out.push_back(st[a]);
        st.swap(out);
    }
}

bool make_quads(const Table &t, std::vector<int> &out) {
    out.clear();
    if (t.size() < 2) return false;
    const int np = (int)t[0].size();
    std::vector<int> owner(2 * np, -1);
    for (size_t s = 0; s + 1 < t.size(); ++s) {
        const Step &cur = t[s], &nxt = t[s + 1];
        if ((int)cur.size() != np || (int)nxt.size() != np) return false;
        for (int i = 0; i < np; ++i) owner[cur[i].first] = owner[cur[i].second] = i;
        std::vector<char> done(np, 0);
        for (int j = 0; j < np; ++j) {
            const int ia = owner[nxt[j].first], ib = owner[nxt[j].second];
            if (ia == ib || ia < 0 || ib < 0) return false;
            if (done[j]) continue;
            // the other new pair of the group must take the other two blocks
            const int a0 = nxt[j].first, b0 = nxt[j].second;
            const int a1 = cur[ia].first == a0 ? cur[ia].second : cur[ia].first;
            const int b1 = cur[ib].first == b0 ? cur[ib].second : cur[ib].first;
            int jy = -1;
            for (int k = 0; k < np; ++k)
                if ((nxt[k].first == a1 && nxt[k].second == b1) ||
                    (nxt[k].first == b1 && nxt[k].second == a1))
                    jy = k;
            if (jy < 0 || jy == j) return false;
            done[j] = done[jy] = 1;
            const int q[8] = {ia, ib, j, jy, a0, b0, 0, 0};
            out.insert(out.end(), q, q + 8);
        }
    }
    return true;
}

}  // namespace jsvd
