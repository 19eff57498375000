"""Pins for the strategy oracle (Section 3): hand-derived tables, Lemma 3.2,
the p-strategy definition (3.1), and the paper's statements about
Algorithm 3.2 and the power-of-two orders."""
import os

import pytest

from oracle import strategy as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pstrategies.txt")


def _golden():
    tabs, cur = {}, None
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if "," not in line:
                cur = line
                tabs[cur] = []
                continue
            tabs[cur].append([tuple(int(x) for x in p.split(",")) for p in line.split()])
    return tabs


def _expand(steps, kind):
    """Algorithm 3.2, written here only to check the paper's claim that it
    reproduces Algorithm 3.1 at twice the order."""
    n = 2 * (len(steps) + 1)
    out = [[(2 * k - 1, 2 * k) for k in range(1, n // 2 + 1)]]
    for i in range(2, n):
        cur = []
        for (p, q) in steps[i // 2 - 1]:
            if i % 2 == 0:
                cur += [(2 * p - 1, 2 * q - 1), (2 * p, 2 * q)]
            elif kind == "R":
                cur += [(2 * p - 1, 2 * q), (2 * p, 2 * q - 1)]
            else:
                cur += [(2 * p, 2 * q - 1), (2 * p - 1, 2 * q)]
        out.append(cur)
    return out


@pytest.mark.parametrize("name", ["R4", "R6", "C6", "R8"])
def test_golden_tables(name):
    tabs = _golden()
    n = int(name[1:])
    assert st.closest_pstrategy(n, name[0]) == tabs[name]


@pytest.mark.parametrize("kind", ["R", "C"])
@pytest.mark.parametrize("n", [2, 4, 6, 8, 10, 12, 14, 16, 18, 20])
def test_lemma_3_2_and_validity(kind, n):
    s = st.closest_pstrategy(n, kind)
    assert s[0] == [(2 * k - 1, 2 * k) for k in range(1, n // 2 + 1)]
    assert st.is_pstrategy(s, n)
    r = st.reverse(s)
    assert st.is_pstrategy(r, n)
    assert r[-1] == list(reversed(s[0]))


@pytest.mark.parametrize("kind", ["R", "C"])
@pytest.mark.parametrize("n", [4, 6, 8, 10, 12])
def test_expansion_equals_closest(kind, n):
    """Section 3: the expansion of O_n equals O_2n for the orders checked."""
    assert _expand(st.closest_pstrategy(n, kind), kind) == st.closest_pstrategy(2 * n, kind)


@pytest.mark.parametrize("n", [4, 8, 16, 32])
def test_power_of_two_no_backtracking(n):
    r, stats = st.closest_pstrategy(n, "R", return_stats=True)
    c, stats_c = st.closest_pstrategy(n, "C", return_stats=True)
    assert stats["backtracks"] == 0 and stats_c["backtracks"] == 0
    # R and C are step-equivalent for these orders
    assert [sorted(x) for x in r] == [sorted(x) for x in c]


def test_invalid_detected():
    s = st.closest_pstrategy(6, "R")
    bad = [list(x) for x in s]
    bad[1][0], bad[2][0] = bad[2][0], bad[1][0]
    assert st.is_pstrategy(s, 6)
    assert not st.is_pstrategy([s[0]] * 5, 6)


@pytest.mark.parametrize("name", ["RR4", "RR6"])
def test_round_robin_golden(name):
    tabs = _golden()
    assert st.round_robin(int(name[2:])) == tabs[name]


@pytest.mark.parametrize("n", [2, 4, 6, 8, 10, 16, 22, 64, 128, 130])
def test_round_robin_is_pstrategy(n):
    s = st.round_robin(n)
    assert st.is_pstrategy(s, n)
    assert s[0] == [(2 * k - 1, 2 * k) for k in range(1, n // 2 + 1)]
