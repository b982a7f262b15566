"""Writes step_examples.json: worked examples of the step-function local constants of Sec. 4.3.

The paper describes M_k(t) in words only and prints no numbers, so every
table and bound below is worked by hand (the comments show the work) under
the reading stated in the oracle: knots q_1..q_K shared by all data; for datum
k, d1 = distance to the nearest other datum, V_0 = largest slope among the
data at distance <= d1, V_s = largest slope among the data at distance
<= max(q_s, d1), V_{K+1} = largest slope overall; M_k(t) = V_0 for t <= d1,
else V_s for the first knot with t <= q_s, else V_{K+1}; bounds of Eq. (2)
with M_k(dist) in place of M.  The script re-derives each hand value from
that reading in exact rationals (``fractions``) to guard the literals
against typos; nothing here calls the oracle or the GPU library.
Run:  python tests/golden/make_step_examples.py
"""
import json
import os
from fractions import Fraction as F

HERE = os.path.dirname(os.path.abspath(__file__))


def isqrt_exact(v: F) -> F:
    """Square root of a rational that is a perfect square (asserted)."""
    import math
    n, d = v.numerator, v.denominator
    rn, rd = math.isqrt(n), math.isqrt(d)
    assert rn * rn == n and rd * rd == d, f"{v} is not a perfect square"
    return F(rn, rd)


def dist(a, b, norm, mon=None, up=True):
    comps = []
    for i, (ai, bi) in enumerate(zip(a, b)):
        dlt = ai - bi
        m = 0 if mon is None else mon[i]
        if m == 0:
            c = abs(dlt)
        elif (m > 0) == up:
            c = max(dlt, F(0))
        else:
            c = max(-dlt, F(0))
        comps.append(c)
    if norm == "l1":
        return sum(comps, F(0))
    if norm == "linf":
        return max(comps)
    return isqrt_exact(sum((c * c for c in comps), F(0)))


def table(x, y, knots, norm):
    n, K = len(x), len(knots)
    d1s, Vs = [], []
    for k in range(n):
        pairs = [(dist(x[k], x[j], norm), abs(y[k] - y[j])) for j in range(n) if j != k]
        pairs = [(t, dy / t) for t, dy in pairs if t > 0]
        d1 = min(t for t, _ in pairs)
        rads = [d1] + [max(q, d1) for q in knots] + [None]
        V = [max([s for t, s in pairs if rad is None or t <= rad] + [F(0)]) for rad in rads]
        d1s.append(d1)
        Vs.append(V)
    return d1s, Vs


def step(t, d1, V, knots):
    if t <= d1:
        return V[0]
    for s, q in enumerate(knots, start=1):
        if t <= q:
            return V[s]
    return V[-1]


def bounds(x, y, knots, d1, V, q, norm, mon):
    us = [y[k] + step(dist(q, x[k], norm, mon, True), d1[k], V[k], knots) *
          dist(q, x[k], norm, mon, True) for k in range(len(x))]
    ls = [y[k] - step(dist(q, x[k], norm, mon, False), d1[k], V[k], knots) *
          dist(q, x[k], norm, mon, False) for k in range(len(x))]
    hu, hl = min(us), max(ls)
    return hu, hl, us.index(hu), ls.index(hl)


def s(v):
    return str(v)


def case_1d():
    # x = 0, 1, 3, 6 with y = 0, 1, 4, 10; knots 3/2, 4.  Slopes: (0,1) 1,
    # (0,3) 4/3, (0,6) 5/3, (1,3) 3/2, (1,6) 9/5, (3,6) 2.
    #   k=0: d1 = 1;  V0 {1}: 1;  V1 r=3/2 {1}: 1;  V2 r=4 {1, 3}: 4/3;  V3: 5/3
    #   k=1: d1 = 1;  V0 {0}: 1;  V1: 1;  V2 r=4 {0, 3}: 3/2;  V3: 9/5
    #   k=2: d1 = 2;  V0 {1}: 3/2;  V1 r=max(3/2,2)=2: 3/2;  V2 r=4 {0,1,6}: 2;  V3: 2
    #   k=3: d1 = 3;  V0 {3}: 2;  V1 r=3: 2;  V2 r=4 {3}: 2;  V3: 2
    x = [[F(0)], [F(1)], [F(3)], [F(6)]]
    y = [F(0), F(1), F(4), F(10)]
    knots = [F(3, 2), F(4)]
    d1 = [F(1), F(1), F(2), F(3)]
    V = [[F(1), F(1), F(4, 3), F(5, 3)], [F(1), F(1), F(3, 2), F(9, 5)],
         [F(3, 2), F(3, 2), F(2), F(2)], [F(2), F(2), F(2), F(2)]]
    # queries (distances t to the four data, M_k(t), u, l):
    #   x = 2:   t 2,1,1,4  M 4/3,1,3/2,2  u 8/3,2,11/2,18  l -8/3,0,5/2,2
    #            H_up 2 (k=1), H_lo 5/2 (k=2)
    #   x = 1/2: t 1/2,1/2,5/2,11/2  M 1,1,2,2  u 1/2,3/2,9,21  l -1/2,1/2,-1,-1
    #            H_up 1/2 (k=0), H_lo 1/2 (k=1)
    #   x = 7:   t 7,6,4,1  M 5/3,9/5,2,2  u 35/3,59/5,12,12  l -35/3,-49/5,-4,8
    #            H_up 35/3 (k=0), H_lo 8 (k=3)
    #   x = 1:   t 1,0,2,5  M 1,1,3/2,2  u 1,1,7,20  l -1,1,1,0
    #            H_up 1 (k=0, tie with k=1), H_lo 1 (k=1, tie with k=2)
    # distances exactly at a knot take that knot's segment (t <= q_s):
    #   x = -4:  t 4,5,7,10  M 4/3,9/5,2,2  u 16/3,10,18,30  l -16/3,-8,-10,-10
    #            H_up 16/3 (k=0), H_lo -16/3 (k=0)
    #   x = 5/2: t 5/2,3/2,1/2,7/2  M 4/3,1,3/2,2  u 10/3,5/2,19/4,17  l -10/3,-1/2,13/4,3
    #            H_up 5/2 (k=1), H_lo 13/4 (k=2)
    queries = [([F(2)], F(2), F(5, 2), 1, 2), ([F(1, 2)], F(1, 2), F(1, 2), 0, 1),
               ([F(7)], F(35, 3), F(8), 0, 3), ([F(1)], F(1), F(1), 0, 1),
               ([F(-4)], F(16, 3), F(-16, 3), 0, 0), ([F(5, 2)], F(5, 2), F(13, 4), 1, 2)]
    out = []
    for norm in ("l1", "l2", "linf"):  # one coordinate: every norm is |.|
        assert table(x, y, knots, norm) == (d1, V)
        qs = []
        for q, hu, hl, au, al in queries:
            assert bounds(x, y, knots, d1, V, q, norm, None) == (hu, hl, au, al)
            qs.append(dict(xq=[s(v) for v in q], h_up=s(hu), h_lo=s(hl), g=s((hu + hl) / 2),
                           arg_up=au, arg_lo=al))
        out.append(dict(name=f"1d_{norm}", cite="Sec. 4.3, Eq. (2)", norm=norm, mon=None,
                        x=[[s(v) for v in r] for r in x], y=[s(v) for v in y],
                        knots=[s(v) for v in knots], d1=[s(v) for v in d1],
                        V=[[s(v) for v in r] for r in V], queries=qs))
    return out


def case_2d_l2():
    # 3-4-5 geometry: x = (0,0), (3,4), (6,0), (0,8), y = 0, 5, 3, 16, l2,
    # knots 11/2, 9.  Distances and slopes: (0,1) 5, 1; (0,2) 6, 1/2;
    # (0,3) 8, 2; (1,2) 5, 2/5; (1,3) 5, 11/5; (2,3) 10, 13/10.
    #   k=0: d1 5; V0 1; V1 r=11/2 {1}: 1; V2 r=9 {1,2,3}: 2; V3 2
    #   k=1: d1 5 (three at 5); V0 11/5; V1 11/5; V2 11/5; V3 11/5
    #   k=2: d1 5; V0 2/5; V1 2/5; V2 r=9 {0,1}: 1/2; V3 13/10
    #   k=3: d1 5; V0 11/5; V1 11/5; V2 r=9 {0,1}: 11/5; V3 11/5
    x = [[F(0), F(0)], [F(3), F(4)], [F(6), F(0)], [F(0), F(8)]]
    y = [F(0), F(5), F(3), F(16)]
    knots = [F(11, 2), F(9)]
    d1 = [F(5)] * 4
    V = [[F(1), F(1), F(2), F(2)], [F(11, 5)] * 4, [F(2, 5), F(2, 5), F(1, 2), F(13, 10)],
         [F(11, 5)] * 4]
    assert table(x, y, knots, "l2") == (d1, V)
    return dict(name="2d_l2_table", cite="Sec. 4.3", norm="l2", mon=None,
                x=[[s(v) for v in r] for r in x], y=[s(v) for v in y],
                knots=[s(v) for v in knots], d1=[s(v) for v in d1],
                V=[[s(v) for v in r] for r in V], queries=[])


def case_2d_l1_monotone():
    # x = (0,0), (1,0), (3,2), y = 0, 2, 3, l1, one knot 2.  Symmetric
    # distances and slopes: (0,1) 1, 2; (0,2) 5, 3/5; (1,2) 4, 1/4.
    #   k=0: d1 1; V0 2; V1 r=2 {1}: 2; V2 2
    #   k=1: d1 1; V0 2; V1 2; V2 2
    #   k=2: d1 4; V0 1/4; V1 r=max(2,4)=4: 1/4; V2 3/5
    # Bounds with coordinate 0 increasing (Eq. 4 for the upper distance, its
    # mirror for the lower one):
    #   query (2,1): up distances 3, 2, 1; lo distances 1, 1, 2
    #     u: 0+2*3=6, 2+2*2=6, 3+1/4=13/4;  l: 0-2=-2, 2-2=0, 3-1/2=5/2
    #     H_up 13/4 (k=2), H_lo 5/2 (k=2)
    #   query (0,1): up 1, 1, 1; lo 1, 2, 4
    #     u: 2, 4, 13/4;  l: -2, 2-4=-2, 3-1=2
    #     H_up 2 (k=0), H_lo 2 (k=2)
    # the two distances of one pair fall in different segments:
    #   query (-2,2): up 2, 2, 0; lo 4, 5, 5
    #     k=2: M(0) = V0 = 1/4, M(5) = V2 = 3/5
    #     u: 0+4=4, 2+4=6, 3;  l: 0-8=-8, 2-10=-8, 3-3=0
    #     H_up 3 (k=2), H_lo 0 (k=2)
    x = [[F(0), F(0)], [F(1), F(0)], [F(3), F(2)]]
    y = [F(0), F(2), F(3)]
    knots = [F(2)]
    mon = [1, 0]
    d1 = [F(1), F(1), F(4)]
    V = [[F(2)] * 3, [F(2)] * 3, [F(1, 4), F(1, 4), F(3, 5)]]
    assert table(x, y, knots, "l1") == (d1, V)
    queries = [([F(2), F(1)], F(13, 4), F(5, 2), 2, 2), ([F(0), F(1)], F(2), F(2), 0, 2),
               ([F(-2), F(2)], F(3), F(0), 2, 2)]
    qs = []
    for q, hu, hl, au, al in queries:
        assert bounds(x, y, knots, d1, V, q, "l1", mon) == (hu, hl, au, al)
        qs.append(dict(xq=[s(v) for v in q], h_up=s(hu), h_lo=s(hl), g=s((hu + hl) / 2),
                       arg_up=au, arg_lo=al))
    return dict(name="2d_l1_monotone", cite="Sec. 4.3, Eq. (2), Eq. (4)", norm="l1", mon=mon,
                x=[[s(v) for v in r] for r in x], y=[s(v) for v in y],
                knots=[s(v) for v in knots], d1=[s(v) for v in d1],
                V=[[s(v) for v in r] for r in V], queries=qs)


def main():
    cases = case_1d() + [case_2d_l2(), case_2d_l1_monotone()]
    with open(os.path.join(HERE, "step_examples.json"), "w") as f:
        json.dump(dict(source="worked by hand from Sec. 4.3 and Eq. (2); see make_step_examples.py",
                       cases=cases), f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
