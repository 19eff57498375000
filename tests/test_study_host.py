"""Host logic of the strategy/variant study (no GPU): the case list and the
table rendering."""
from paper_1401_2720_amd import study


def test_quick_cases_and_table():
    cases = study._cases(quick=True)
    assert [c[0] for c in cases] == ["graded256"]
    assert len(study._cases(quick=False)) == 4
    rows = [dict(input="x", w=16, inner="block-oriented", strategy=s, sweeps=3, converged=1,
                 rotations=10, inner_sweeps=5, seconds=0.5, sigma_dev=0.0)
            for s in study.STRATEGIES]
    t = study.table(rows).splitlines()
    assert len(t) == 2 + len(rows)
    assert t[2].startswith("| x | 16 | block-oriented | rrev | 3 | 10 | 5 | 0.500 |")
