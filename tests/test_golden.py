"""The oracle against hand-worked examples (tests/golden/): every
displacement's N and joint counts exactly, MI within 1e-14 of the closed
form derived on paper from Eq. 1 / Eq. 5, and Alg. 1's choice (threshold,
argmax, ties to the smallest row-major index).  Each fixture is also checked
against itself: its listed counts must give its closed-form MI by Eq. 1, and
its N must be the sum of its counts, so a slip in a fixture cannot pass."""

import numpy as np
import pytest

import golden_io

MI_CLOSED_TOL = 1e-14


@pytest.mark.parametrize("name", golden_io.fixtures())
def test_fixture_is_consistent(name):
    fx = golden_io.load(name)
    ha, wa = fx["A"].shape
    hb, wb = fx["B"].shape
    seen = {(s["dy"], s["dx"]) for s in fx["shifts"]}
    # every displacement of the (H_A + H_B - 1) x (W_A + W_B - 1) map once
    assert len(seen) == len(fx["shifts"]) == (ha + hb - 1) * (wa + wb - 1)
    for s in fx["shifts"]:
        assert -(ha - 1) <= s["dy"] <= hb - 1 and -(wa - 1) <= s["dx"] <= wb - 1
        assert s["joint"].sum() == s["n"], s
        assert abs(golden_io.mi_of_counts(s["joint"]) - s["mi"]) <= MI_CLOSED_TOL, s


@pytest.mark.parametrize("name", golden_io.fixtures())
def test_oracle_matches_worked_example(oracle, name):
    fx = golden_io.load(name)
    qa, qb = fx["qa"], fx["qb"]
    o = oracle.cmif_direct(fx["A"], fx["MA"], fx["B"], fx["MB"], qa, qb,
                           counts=True)
    ha, wa = fx["A"].shape
    sw = o["mi"].shape[1]
    for s in fx["shifts"]:
        i, j = s["dy"] + ha - 1, s["dx"] + wa - 1
        assert o["n"][i, j] == s["n"], s
        assert np.array_equal(o["counts"][:, :, i, j], s["joint"]), s
        assert abs(o["mi"][i, j] - s["mi"]) <= MI_CLOSED_TOL, (s, o["mi"][i, j])
    for g in fx["argmax"]:
        idx, _, _ = oracle.argmax(o["mi"], o["n"], g["gamma"])
        assert divmod(idx, sw) == (g["dy"] + ha - 1, g["dx"] + wa - 1), g


# --- spatially weighted MI (Sec. 3.3, Eq. 13) -------------------------------

def _memberships(labels, weights, q):
    """Weighted level sets of Eq. 13: plane a holds W(x) where the label is a."""
    return np.stack([(labels == a) * weights for a in range(q)]).astype(np.float32)


@pytest.mark.parametrize("name", golden_io.fixtures("swmi"))
def test_swmi_fixture_is_consistent(name):
    fx = golden_io.load(name)
    ha, wa = fx["A"].shape
    hb, wb = fx["B"].shape
    assert len({(s["dy"], s["dx"]) for s in fx["shifts"]}) == len(fx["shifts"]) \
        == (ha + hb - 1) * (wa + wb - 1)
    for s in fx["shifts"]:
        assert s["joint"].sum() == s["n"], s
        assert abs(golden_io.mi_of_counts(s["joint"]) - s["mi"]) <= MI_CLOSED_TOL, s


@pytest.mark.parametrize("name", golden_io.fixtures("swmi"))
def test_soft_oracles_match_worked_swmi(oracle, name):
    """The C direct soft method (weighted joints exactly, MI to 1e-14) and
    the FP64 torch FFT formulation behind the gradient tests (to 1e-12)."""
    import torch
    fx = golden_io.load(name)
    qa, qb = fx["qa"], fx["qb"]
    pa = _memberships(fx["A"], fx["WA"], qa)
    pb = _memberships(fx["B"], fx["WB"], qb)
    ones_a = np.ones(fx["A"].shape, np.uint8)
    ones_b = np.ones(fx["B"].shape, np.uint8)
    o = oracle.soft_direct(pa, ones_a, pb, ones_b, joint=True)
    jt = oracle.soft_joint_torch(torch.from_numpy(pa).double(),
                                 torch.ones(fx["A"].shape, dtype=torch.float64),
                                 torch.from_numpy(pb).double(),
                                 torch.ones(fx["B"].shape, dtype=torch.float64))
    mt, nt = oracle.soft_mi_torch(jt)
    ha, wa = fx["A"].shape
    for s in fx["shifts"]:
        i, j = s["dy"] + ha - 1, s["dx"] + wa - 1
        assert o["n"][i, j] == s["n"], s
        assert np.array_equal(o["joint"][:, :, i, j], s["joint"].astype(np.float64)), s
        assert abs(o["mi"][i, j] - s["mi"]) <= MI_CLOSED_TOL, (s, o["mi"][i, j])
        assert abs(float(nt[i, j]) - s["n"]) <= 1e-12, s
        assert abs(float(mt[i, j]) - s["mi"]) <= 1e-12, (s, float(mt[i, j]))
