"""Pins for the dynamic-offset neighbourhood (Sec. 4.2, Sec. 5.2).

The per-case cell counts and the average count are the paper's printed
values; coverage is checked by locating random displaced points in the
rearranged, tiled space and requiring their (cell, image) to be listed.
"""
import numpy as np
import pytest

from test_oracle_forces import read_golden


def generic_R(l, rc, seed):
    g = np.random.default_rng(seed)
    w = rc * (1.0 + g.uniform(0.05, 0.4, size=3))
    r = w * np.asarray(l)
    R = np.diag(r)
    R[0, 1] = g.uniform(0, r[0])      # r12
    R[0, 2] = g.uniform(0, r[0])      # r13
    R[1, 2] = g.uniform(0, r[1])      # r23
    return R


def face_case(b, c, l):
    on_xz = b in (0, l[1] - 1)
    on_xy = c in (0, l[2] - 1)
    return {(False, False): "interior", (True, False): "xz", (False, True): "xy", (True, True): "both"}[(on_xz, on_xy)]


@pytest.mark.parametrize("seed", range(5))
def test_case_counts_and_average(orc, seed):
    gold = read_golden()
    expect = {"interior": gold["do_cells_interior"], "xz": gold["do_cells_xz_face"],
              "xy": gold["do_cells_xy_face"], "both": gold["do_cells_both_faces"]}
    l = [5 + seed % 3, 4 + seed, 6 + (seed * 7) % 5]
    rc = 1.0
    R = generic_R(l, rc, seed)
    total = 0
    for c in range(l[2]):
        for b in range(l[1]):
            for a in range(l[0]):
                nb = orc.do_neighbourhood(R, l, rc, a, b, c)
                assert len(nb) == expect[face_case(b, c, l)], (a, b, c)
                # every (cell, image) entry is distinct
                assert len({tuple(r) for r in nb.tolist()}) == len(nb)
                total += len(nb)
    avg = total / (l[0] * l[1] * l[2])
    l2, l3 = l[1], l[2]
    assert abs(avg - (27 + 14 / l3 + 6 / l2 - 4 / (l2 * l3))) < 1e-12


def locate(R, l, p):
    """Cell and lattice image of an arbitrary point in the rearranged tiling."""
    w = np.diag(R) / np.asarray(l)
    y = p.copy()
    k = int(np.floor(y[2] / R[2, 2]))
    y -= k * R[:, 2]
    j = int(np.floor(y[1] / R[1, 1]))
    y -= j * R[:, 1]
    i = int(np.floor(y[0] / R[0, 0]))
    y -= i * R[:, 0]
    cell = np.minimum(np.floor(y / w).astype(int), np.asarray(l) - 1)
    return (int(cell[0]), int(cell[1]), int(cell[2]), i, j, k)


@pytest.mark.parametrize("seed", range(4))
def test_neighbourhood_covers_cutoff_sphere(orc, seed):
    g = np.random.default_rng(50 + seed)
    l = [3 + seed, 4, 3 + (seed % 2)]
    rc = 1.3
    R = generic_R(l, rc, seed + 10)
    if seed == 3:                     # aligned faces (planar flow: r13 = r23 = 0)
        R[0, 2] = R[1, 2] = 0.0
    w = np.diag(R) / np.asarray(l)
    for _ in range(3000):
        a, b, c = (int(g.integers(0, l[0])), int(g.integers(0, l[1])), int(g.integers(0, l[2])))
        p = (np.array([a, b, c]) + g.uniform(0, 1, 3)) * w
        d = g.normal(size=3)
        d *= rc * g.uniform(0, 1) ** (1 / 3) / np.linalg.norm(d)
        nb = {tuple(r) for r in orc.do_neighbourhood(R, l, rc, a, b, c).tolist()}
        nt = {tuple(r) for r in orc.do_neighbourhood(R, l, rc, a, b, c, tight=True).tolist()}
        assert nt <= nb
        assert locate(R, l, p + d) in nt


def test_aligned_layers_need_no_expansion(orc):
    # with r13 = r23 = 0 (planar flow) the z-crossing layer is not offset, so
    # only rows crossing a y face grow: the average is 27 + 6 / l2
    l = [6, 5, 7]
    R = generic_R(l, 1.0, 3)
    R[0, 2] = R[1, 2] = 0.0
    tot = sum(len(orc.do_neighbourhood(R, l, 1.0, a, b, c, tight=False))
              for a in range(l[0]) for b in range(l[1]) for c in range(l[2]))
    assert abs(tot / np.prod(l) - (27 + 6 / l[1])) < 1e-12


def test_two_dimensional_top_row_count(orc):
    """Sec. 4.2, 2-D discussion: a cell in the top row of a rectangular box
    whose top neighbours are shifted by the face offset needs ten cells (the
    crossing row overlaps four cells).  With r13 = r23 = 0 every z layer is
    this 2-D case: the home layer of a top-row cell holds ten (cell, image)
    entries, an interior row's nine."""
    gold = read_golden()
    l = [6, 5, 7]
    R = generic_R(l, 1.0, 4)
    R[0, 2] = R[1, 2] = 0.0
    c = 3
    for a in range(l[0]):
        for b, expect in ((l[1] - 1, gold["do_2d_top_row_cells"]), (0, gold["do_2d_top_row_cells"]), (2, 9)):
            nb = orc.do_neighbourhood(R, l, 1.0, a, b, c)
            layer = nb[(nb[:, 2] == c) & (nb[:, 5] == 0)]
            assert len(layer) == expect, (a, b, len(layer))
