"""Host model of the 2D strip kernels' lane-to-column mapping (csrc/step2d.hpp).

Checks, for every supported cells-per-lane width, both boundary kinds and
ragged widths, that every load stays inside the row and is vector-aligned,
that every cell is written by exactly one lane, and that every written cell's
stencil operands are the right columns: its x neighbours in the one-step
strip, and in the two-step strip the step-1 values (column labels) of the
cell and its neighbours -- including the mirror copies made at no-flux edges.
Also the two-step strip's row schedule, upward and (odd segments) downward:
each row update sees the rows it needs, and every row is written once.
"""
import pytest

W1, W2 = 62, 60  # written lanes per one-step / two-step strip wave


def gmap(i, n, periodic):
    if periodic:
        return i % n
    return 0 if i < 0 else (n - 1 if i >= n else i)


def vec_width(nx, elem, cap):
    v = 16 // elem
    while cap > 0 and v > cap:
        v //= 2
    while v > 1:
        if nx % v == 0:
            return v
        v //= 2
    return 1


def neighbour(arr, lane, i, d, V):
    """Slot value left (d < 0) or right of (lane, i), lanes rotating as in the kernels."""
    if d < 0:
        return arr[lane][i - 1] if i > 0 else arr[(lane - 1) % 64][V - 1]
    return arr[lane][i + 1] if i + 1 < V else arr[(lane + 1) % 64][0]


def one_step(nx, V, per):
    written = [0] * nx
    for tx in range((nx + W1 * V - 1) // (W1 * V)):
        held = []
        for lane in range(64):
            cs = (tx * W1 - 1 + lane) * V
            col, fixL, fixR = cs, False, False
            if cs < 0:
                col, fixL = (nx - V if per else 0), not per
            elif cs >= nx:
                col, fixR = (0 if per else nx - V), not per
            assert 0 <= col <= nx - V and col % V == 0
            slots = [col + i for i in range(V)]
            if V > 1 and fixL:
                slots[V - 1] = slots[0]
            if V > 1 and fixR:
                slots[0] = slots[V - 1]
            held.append(slots)
        for lane in range(1, W1 + 1):
            cs = (tx * W1 - 1 + lane) * V
            if cs >= nx:
                continue
            for i in range(V):
                X = cs + i
                written[X] += 1
                assert held[lane][i] == X
                assert neighbour(held, lane, i, -1, V) == gmap(X - 1, nx, per)
                assert neighbour(held, lane, i, +1, V) == gmap(X + 1, nx, per)
    assert written == [1] * nx


def two_steps(nx, V, per):
    written = [0] * nx
    for tx in range((nx + W2 * V - 1) // (W2 * V)):
        s0, fix = [], []
        for lane in range(64):
            cs = (tx * W2 - 2 + lane) * V
            fixL = fixR = False
            if per:
                col = cs % nx
            elif 0 <= cs < nx:
                col = cs
            elif cs == -V:
                col, fixL = 0, True
            elif cs == nx:
                col, fixR = nx - V, True
            else:
                col = 0 if cs < 0 else nx - V
            assert 0 <= col <= nx - V and col % V == 0
            slots = [col + i for i in range(V)]
            if V > 1 and fixL:
                slots[V - 1] = slots[0]
            if V > 1 and fixR:
                slots[0] = slots[V - 1]
            s0.append(slots)
            fix.append((fixL, fixR))
        # step 1: the column whose one-step stencil a slot evaluated, else None
        s1 = [[X if (neighbour(s0, l, i, -1, V) == gmap(X - 1, nx, per)
                     and neighbour(s0, l, i, +1, V) == gmap(X + 1, nx, per)) else None
               for i, X in enumerate(s0[l])] for l in range(64)]
        c1 = [r[:] for r in s1]  # mirror copies at no-flux edges
        for l in range(64):
            if fix[l][0]:
                c1[l][V - 1] = s1[(l + 1) % 64][0]
            if fix[l][1]:
                c1[l][0] = s1[(l - 1) % 64][V - 1]
        for lane in range(2, W2 + 2):
            cs = (tx * W2 - 2 + lane) * V
            if cs >= nx:
                continue
            for i in range(V):
                X = cs + i
                written[X] += 1
                assert c1[lane][i] == X
                assert neighbour(c1, lane, i, -1, V) == gmap(X - 1, nx, per)
                assert neighbour(c1, lane, i, +1, V) == gmap(X + 1, nx, per)
    assert written == [1] * nx


WIDTHS = list(range(1, 40)) + [60, 61, 62, 63, 64, 119, 120, 121, 124, 125, 240, 241, 248, 250,
                              256, 300, 496, 512, 1000, 1024]


@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("elem,cap", [(8, 1), (8, 2), (4, 1), (4, 2), (4, 4)])
def test_strip_lane_mapping(elem, cap, periodic):
    for nx in WIDTHS:
        V = vec_width(nx, elem, cap)
        one_step(nx, V, periodic)
        two_steps(nx, V, periodic)


def two_step_rows(ny, m0, m1, per, down):
    """Row schedule of the two-step strip (strip2d_x2) over rows m0..m1-1, marching up or, for
    odd segments, down: checks that every step-1 row update sees the state rows it needs in its
    window (the row itself, the next row of the march, and the row before it for the carried
    face), every step-2 update the step-1 rows it needs, and returns the rows written."""
    d = -1 if down else 1
    top = not per and m0 == 0
    bot = not per and m1 == ny
    first_edge = bot if down else top

    def rowmap(s):
        return s % ny if per else min(max(s, 0), ny - 1)

    r_first = (ny - 1 if bot else m1) if down else (0 if top else m0 - 1)
    win = {"prev": rowmap(r_first - d), "cur": rowmap(r_first), "next": rowmap(r_first + d),
           "ahead": rowmap(r_first + 2 * d)}

    def step1(r):
        assert per or 0 <= r < ny, ("step-1 row outside the grid", r)
        assert win["cur"] == rowmap(r) and win["next"] == rowmap(r + d) and win["prev"] == rowmap(r - d), r
        win["prev"], win["cur"], win["next"] = win["cur"], win["next"], win["ahead"]
        win["ahead"] = rowmap(r + 3 * d)
        return ("s1", rowmap(r))  # step-1 value of that row (a mirror ghost is the same record)

    written = []
    outer = step1(r_first)
    c1 = outer if first_edge else step1(r_first + d)
    k1 = outer

    def step2(q):
        nonlocal c1, k1
        assert c1 == ("s1", rowmap(q)) and n1[0] == ("s1", rowmap(q + d)) and k1 == ("s1", rowmap(q - d)), q
        written.append(q)
        k1, c1 = c1, n1[0]

    n1 = [None]
    q0, qlast = (m1 - 1, m0) if down else (m0, m1 - 1)
    q = q0
    while q != qlast:
        n1[0] = step1(q + d)
        step2(q)
        q += d
    last_edge = top if down else bot
    n1[0] = c1 if last_edge else step1(qlast + d)
    step2(qlast)
    return written


@pytest.mark.parametrize("periodic", [False, True])
def test_two_step_row_schedule_both_directions(periodic):
    for ny in range(1, 14):
        for seg in range(1, 6):
            written = []
            for sg, m0 in enumerate(range(0, ny, seg)):
                m1 = min(m0 + seg, ny)
                rows = two_step_rows(ny, m0, m1, periodic, down=bool(sg & 1))
                assert sorted(rows) == list(range(m0, m1))
                assert rows == (list(range(m1 - 1, m0 - 1, -1)) if sg & 1 else list(range(m0, m1)))
                written += rows
            assert sorted(written) == list(range(ny)), (ny, seg)
