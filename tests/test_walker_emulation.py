"""CPU emulation of the unit walker of the row kernel (mv_rows_kernel):
one wavefront walks its share of a segment's leaves as a stream of (leaf,
column pass) units through a ring of D register slots: D - 1 units are
issued before the loop, then each iteration issues one more unit, adds the
oldest one and shifts the ring; a leaf with no columns still issues one
(empty) unit.  The emulation follows the kernel's control flow statement
by statement and checks, over random leaf lists (1..64 leaves per wave,
0..70 columns per leaf, every column-pass width the quad layout produces),
that every issued unit is added exactly once and in order, and that the
result equals the direct product, for every ring depth D >= 2.  With
D = 1 nothing is issued before the loop and every contribution is dropped,
which the kernel now rejects at compile time."""
import numpy as np
import pytest


def walk(ncols, width, D):
    """Units added by the walker, in order: (leaf, first column of the pass)."""
    cnt = len(ncols)
    st = {"i": 0, "c0": 0, "more": True, "issued": 0}
    ring = [None] * D

    def issue():
        if not st["more"]:
            return None                      # zero unit, `issued` unchanged
        unit = (st["i"], st["c0"])
        st["issued"] += 1
        st["c0"] += width
        if st["c0"] >= ncols[st["i"]]:
            st["c0"] = 0
            st["i"] += 1
            if st["i"] >= cnt:
                st["more"] = False
        return unit

    for s in range(D - 1):
        ring[s] = issue()
    added = []
    done = 0
    while done < st["issued"]:
        ring[D - 1] = issue()
        if ring[0] is not None:
            added.append(ring[0])
        for s in range(D - 1):
            ring[s] = ring[s + 1]
        done += 1
    return added


def expected_units(ncols, width):
    out = []
    for i, nc in enumerate(ncols):
        for c0 in range(0, max(nc, 1), width):
            out.append((i, c0))
    return out


@pytest.mark.parametrize("D", [2, 3, 4, 6, 8])
def test_every_unit_added_once_in_order(D):
    rng = np.random.default_rng(D)
    for trial in range(400):
        cnt = int(rng.integers(1, 65))
        ncols = [int(v) for v in rng.integers(0, 71, cnt)]
        # width = columns per unit per pass: NC (1 FP64, 2 FP32) x cpp (64 / lanes per column)
        width = int(rng.choice([1, 2])) * int(rng.choice([1, 2, 4, 8, 16, 32, 64]))
        assert walk(ncols, width, D) == expected_units(ncols, width), (D, trial)


@pytest.mark.parametrize("D", [2, 3, 4])
def test_walker_sum_equals_direct_product(D):
    """Rows 4q..4q+3 of a segment: the sum over the added units of the
    unit's columns weighted by w equals the direct product."""
    rng = np.random.default_rng(10 + D)
    R = 16
    for trial in range(100):
        cnt = int(rng.integers(1, 20))
        ncols = [int(v) for v in rng.integers(0, 40, cnt)]
        data = [rng.standard_normal((R, max(nc, 1))) for nc in ncols]
        wts = [rng.standard_normal(max(nc, 1)) for nc in ncols]
        NC, cpp = 2, 4
        acc = np.zeros(R)
        for (i, c0) in walk(ncols, NC * cpp, D):
            for s in range(NC):
                for co in range(cpp):
                    c = c0 + s * cpp + co
                    if c < ncols[i]:
                        acc += data[i][:, c] * wts[i][c]
        ref = sum(data[i][:, :ncols[i]] @ wts[i][:ncols[i]] for i in range(cnt))
        np.testing.assert_allclose(acc, ref, rtol=1e-12, atol=1e-12)


def test_depth_one_drops_every_unit():
    assert walk([5, 3, 9], 4, 1) == []
