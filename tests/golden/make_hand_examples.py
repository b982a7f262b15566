"""Writes hand_examples.json: tiny worked examples of Eqs. (2)-(4) in exact arithmetic.

The paper prints no numeric example, so these cases are worked by hand from
its definitions and evaluated here with exact rationals (``fractions``) from
the closed forms stated next to each case; nothing here calls the oracle or
the GPU library.  Run:  python tests/golden/make_hand_examples.py
"""
import json
import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


def case_1d_three_points():
    # Eq. (2) in one dimension, M = 1, data (0,0), (1,1), (3,0).  Every
    # distance is |x - x^k| (all norms agree in 1-D).  Closed form for each
    # query: compare the three candidates by hand.
    x = [F(0), F(1), F(3)]
    y = [F(0), F(1), F(0)]
    M = F(1)
    queries = [F(2), F(1, 2), F(-1), F(4)]
    # x = 2:   up: 0+2, 1+1, 0+1 -> 1 at k=2;   lo: 0-2, 1-1, 0-1 -> 0 at k=1
    # x = 1/2: up: 1/2, 3/2, 5/2 -> 1/2 at k=0; lo: -1/2, 1/2, -5/2 -> 1/2 at k=1
    # x = -1:  up: 1, 3, 4 -> 1 at k=0;          lo: -1, -1, -4 -> -1 at k=0 (tie, lowest)
    # x = 4:   up: 4, 4, 1 -> 1 at k=2;          lo: -4, -2, -1 -> -1 at k=2
    expect = [
        (F(1), F(0), 2, 1),
        (F(1, 2), F(1, 2), 0, 1),
        (F(1), F(-1), 0, 0),
        (F(1), F(-1), 2, 2),
    ]
    out = []
    for xq, (hu, hl, au, al) in zip(queries, expect):
        # re-derive from the closed form to guard typos in the table above
        cu = [y[k] + M * abs(xq - x[k]) for k in range(3)]
        cl = [y[k] - M * abs(xq - x[k]) for k in range(3)]
        assert min(cu) == hu and cu.index(min(cu)) == au
        assert max(cl) == hl and cl.index(max(cl)) == al
        out.append(dict(xq=[str(xq)], h_up=str(hu), h_lo=str(hl), g=str((hu + hl) / 2),
                        arg_up=au, arg_lo=al))
    return dict(name="1d_three_points", cite="Eq. (2), Eq. (3)", norm="l1", M=str(M),
                mon=[0], x=[[str(v)] for v in x], y=[str(v) for v in y], queries=out)


def case_2d_monotone():
    # Eq. (4): increasing in both coordinates, l1 norm, M = 2, data
    # (0,0)->0, (1,1)->2.  Upper distance ||(x - x^k)_+||_1, lower distance
    # ||(x^k - x)_+||_1 (mirror image of Eq. 4).
    # query (1/2, 1/2): up: 0 + 2*(1/2+1/2) = 2 (k=0), 2 + 2*0 = 2 (k=1) -> 2 at k=0
    #                   lo: 0 - 2*0 = 0 (k=0), 2 - 2*(1/2+1/2) = 0 (k=1) -> 0 at k=0
    # query (2, 0):     up: 0 + 2*2 = 4, 2 + 2*(1+0) = 4 -> 4 at k=0
    #                   lo: 0 - 0 = 0, 2 - 2*(0+1) = 0 -> 0 at k=0
    # query (-1, 3):    up: 0 + 2*3 = 6, 2 + 2*(0+2) = 6 -> 6 at k=0
    #                   lo: 0 - 2*(1+0) = -2, 2 - 2*(2+0) = -2 -> -2 at k=0
    # query (1, 1/4):   up: 0 + 2*(5/4) = 5/2, 2 + 2*0 = 2 -> 2 at k=1
    #                   lo: 0 - 0 = 0, 2 - 2*(0 + 3/4) = 1/2 -> 1/2 at k=1
    x = [(F(0), F(0)), (F(1), F(1))]
    y = [F(0), F(2)]
    M = F(2)
    pos = lambda v: v if v > 0 else F(0)
    queries = [(F(1, 2), F(1, 2)), (F(2), F(0)), (F(-1), F(3)), (F(1), F(1, 4))]
    expect = [(F(2), F(0), 0, 0), (F(4), F(0), 0, 0), (F(6), F(-2), 0, 0), (F(2), F(1, 2), 1, 1)]
    out = []
    for xq, (hu, hl, au, al) in zip(queries, expect):
        cu = [y[k] + M * sum(pos(xq[i] - x[k][i]) for i in range(2)) for k in range(2)]
        cl = [y[k] - M * sum(pos(x[k][i] - xq[i]) for i in range(2)) for k in range(2)]
        assert min(cu) == hu and cu.index(min(cu)) == au
        assert max(cl) == hl and cl.index(max(cl)) == al
        out.append(dict(xq=[str(v) for v in xq], h_up=str(hu), h_lo=str(hl),
                        g=str((hu + hl) / 2), arg_up=au, arg_lo=al))
    return dict(name="2d_monotone_l1", cite="Eq. (2), Eq. (3), Eq. (4)", norm="l1", M=str(M),
                mon=[1, 1], x=[[str(v) for v in p] for p in x], y=[str(v) for v in y],
                queries=out)


def case_2d_linf_local():
    # Eq. (2) with per-datum constants M_k (Sec. 4.3, scalar form), linf norm.
    # data (0,0)->1 with M_0 = 1, (2,0)->0 with M_1 = 1/2.
    # query (1, 1): d_0 = max(1,1) = 1, d_1 = max(1,1) = 1
    #   up: 1 + 1 = 2, 0 + 1/2 = 1/2 -> 1/2 at k=1;  lo: 1 - 1 = 0, 0 - 1/2 = -1/2 -> 0 at k=0
    # query (0, 3): d_0 = 3, d_1 = max(2,3) = 3
    #   up: 4, 3/2 -> 3/2 at k=1;  lo: -2, -3/2 -> -3/2 at k=1
    x = [(F(0), F(0)), (F(2), F(0))]
    y = [F(1), F(0)]
    Mk = [F(1), F(1, 2)]
    queries = [(F(1), F(1)), (F(0), F(3))]
    expect = [(F(1, 2), F(0), 1, 0), (F(3, 2), F(-3, 2), 1, 1)]
    out = []
    for xq, (hu, hl, au, al) in zip(queries, expect):
        dd = [max(abs(xq[i] - x[k][i]) for i in range(2)) for k in range(2)]
        cu = [y[k] + Mk[k] * dd[k] for k in range(2)]
        cl = [y[k] - Mk[k] * dd[k] for k in range(2)]
        assert min(cu) == hu and cu.index(min(cu)) == au
        assert max(cl) == hl and cl.index(max(cl)) == al
        out.append(dict(xq=[str(v) for v in xq], h_up=str(hu), h_lo=str(hl),
                        g=str((hu + hl) / 2), arg_up=au, arg_lo=al))
    return dict(name="2d_linf_local", cite="Eq. (2), Eq. (3), Sec. 4.3", norm="linf", M="0",
                Mk=[str(v) for v in Mk], mon=[0, 0], x=[[str(v) for v in p] for p in x],
                y=[str(v) for v in y], queries=out)


def main():
    cases = [case_1d_three_points(), case_2d_monotone(), case_2d_linf_local()]
    with open(os.path.join(HERE, "hand_examples.json"), "w") as f:
        json.dump(cases, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
