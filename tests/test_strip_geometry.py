"""Host model of the 2D strip kernels' lane-to-column mapping (csrc/step2d.hpp).

Checks, for every supported cells-per-lane width, both boundary kinds and
ragged widths, that every load stays inside the row and is vector-aligned,
that every cell is written by exactly one lane, and that every written cell's
stencil operands are the right columns: its x neighbours in the one-step
strip, and in the two-step strip the step-1 values (column labels) of the
cell and its neighbours -- including the mirror copies made at no-flux edges.
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
