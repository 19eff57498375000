"""Oracle for the parallel pivot strategies of Section 3 (test infrastructure).

Definitions followed:
  * eq. (3.1): for even n a parallel strategy (p-strategy) has s = n - 1
    parallel steps of t = n/2 disjoint pivot pairs, and every pair (i, j),
    1 <= i < j <= n, occurs exactly once per sweep.
  * Definition 3.1: O1 is closer to a sequential strategy O than O2 when the
    sequence of positions (in O) of O1's pairs is lexicographically smaller.
    Within a p-step the pairs are listed by ascending position in O.
  * Algorithm 3.1: the closest p-strategy is found by taking, step after
    step, the lexicographically next set of t disjoint pairs (a maximal
    independent set of the collision graph) among the pairs still unused,
    recursing on the rest, and backtracking when the rest cannot be
    completed.
  * The reverse of a strategy lists its pairs in the opposite order (the
    last pair of the last p-step first).
  * R_n is the row-cyclic order (1,2),(1,3),...,(1,n),(2,3),...;
    C_n is the column-cyclic order (1,2),(1,3),(2,3),(1,4),(2,4),(3,4),...
  * The round-robin ordering (a comparison strategy of Section 6; Brent and
    Luk's parallel ordering): index 1 stays put, the others sit on a ring
    that turns by one place per p-step; see round_robin().

Pairs are one-based (i, j) with i < j, as in the paper.
"""


def sequential_order(n, kind):
    """The sequential cyclic strategy R_n ("R") or C_n ("C") as a list."""
    if kind == "R":
        return [(i, j) for i in range(1, n) for j in range(i + 1, n + 1)]
    if kind == "C":
        return [(i, j) for j in range(2, n + 1) for i in range(1, j)]
    raise ValueError(kind)


class _Search:
    def __init__(self, n, kind, max_nodes):
        self.n = n
        self.t = n // 2
        self.pairs = sequential_order(n, kind)
        self.max_nodes = max_nodes
        self.nodes = 0
        self.backtracks = 0

    def _matchings(self, avail):
        """Yield, in lexicographic order of positions, every set of t
        disjoint pairs drawn from the available positions (sorted list)."""
        n, t, pairs = self.n, self.t, self.pairs
        chosen = []
        covered = [False] * (n + 1)

        def feasible(start):
            # every uncovered index must still be coverable by a later pair
            need = [False] * (n + 1)
            for k in range(start, len(avail)):
                i, j = pairs[avail[k]]
                if not covered[i] and not covered[j]:
                    need[i] = need[j] = True
            return all(covered[i] or need[i] for i in range(1, n + 1))

        def rec(start):
            self.nodes += 1
            if self.max_nodes and self.nodes > self.max_nodes:
                raise RuntimeError("strategy search exceeded its node budget")
            if len(chosen) == t:
                yield list(chosen)
                return
            if not feasible(start):
                return
            for k in range(start, len(avail)):
                i, j = pairs[avail[k]]
                if covered[i] or covered[j]:
                    continue
                covered[i] = covered[j] = True
                chosen.append(avail[k])
                yield from rec(k + 1)
                chosen.pop()
                covered[i] = covered[j] = False

        yield from rec(0)

    def run(self):
        steps = []

        def gen(avail):
            if not avail:
                return True
            for S in self._matchings(avail):
                steps.append(S)
                sset = set(S)
                if gen([a for a in avail if a not in sset]):
                    return True
                steps.pop()
                self.backtracks += 1
            return False

        if not gen(list(range(len(self.pairs)))):
            raise RuntimeError("no p-strategy found")
        return [[self.pairs[k] for k in S] for S in steps]


def closest_pstrategy(n, kind="R", max_nodes=0, return_stats=False):
    """Algorithm 3.1: the p-strategy closest to R_n or C_n (n even)."""
    if n < 2 or n % 2:
        raise ValueError("order must be even and >= 2")
    s = _Search(n, kind, max_nodes)
    steps = s.run()
    if return_stats:
        return steps, dict(backtracks=s.backtracks, nodes=s.nodes)
    return steps


def reverse(steps):
    """The reverse strategy: every pair in the opposite order."""
    return [list(reversed(st)) for st in reversed(steps)]


def is_pstrategy(steps, n):
    """eq. (3.1): n-1 steps of n/2 disjoint pairs covering every pair once."""
    if len(steps) != n - 1:
        return False
    seen = set()
    for st in steps:
        if len(st) != n // 2:
            return False
        idx = [i for p in st for i in p]
        if len(set(idx)) != n:
            return False
        for (i, j) in st:
            if not (1 <= i < j <= n) or (i, j) in seen:
                return False
            seen.add((i, j))
    return len(seen) == n * (n - 1) // 2


def round_robin(n):
    """Round-robin ordering of even order n as p-steps of one-based pairs.

    Index 1 is fixed; the other n - 1 indices sit on a ring, initially
    3, 5, ..., n - 1, n, n - 2, ..., 2, which turns by one place per step
    (entry i of step s is entry i - s of the initial ring, cyclically).
    Step s pairs 1 with the ring's last entry and, for k = 1 .. n/2 - 1,
    ring entry k - 1 with ring entry n - 2 - k (zero-based ring positions),
    in that order; pairs are written (min, max).  Step 0 is (1,2), (3,4), ...
    """
    if n < 2 or n % 2:
        raise ValueError("even order >= 2")
    h = n // 2
    ring0 = list(range(3, n, 2)) + list(range(n, 1, -2))
    L = n - 1
    out = []
    for s in range(n - 1):
        ring = [ring0[(i - s) % L] for i in range(L)]
        step = [tuple(sorted((1, ring[L - 1])))]
        for k in range(1, h):
            step.append(tuple(sorted((ring[k - 1], ring[n - 2 - k]))))
        out.append(step)
    return out
