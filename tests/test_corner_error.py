"""CPU: cmif_corner_error, the success measure of the paper's alignment
experiments (Sec. 5.2: mean distance between the reference image's corners
as landmarks and their recovered positions; success below 2 % of the
width), against closed forms."""

import math

import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def cm():
    import paper_2106_14699_amd as cm
    return cm


def best(angle_index=-1, angle=0.0, dy=0, dx=0):
    return dict(angle_index=angle_index, angle_rad=angle, dy=dy, dx=dx, mi=0.0,
                n=0)


IDENT = (1.0, 0.0, 0.0, 0.0, 1.0, 0.0)


def test_identity_is_zero(cm):
    assert cm.cmif_corner_error(best(), (40, 50, 40, 50), IDENT) == 0.0


def test_translation_error_is_its_length(cm):
    # truth moves every landmark by (3, 4): distance 5 at each corner
    t = (1.0, 0.0, 3.0, 0.0, 1.0, 4.0)
    assert abs(cm.cmif_corner_error(best(), (30, 30, 30, 30), t) - 5.0) < 1e-12
    # a result off by one row from the truth: error 1
    t = (1.0, 0.0, 0.0, 0.0, 1.0, 2.0)
    assert abs(cm.cmif_corner_error(best(0, 0.0, 1, 0), (30, 30, 30, 30), t)
               - 1.0) < 1e-12


@pytest.mark.parametrize("deg", [0.5, 3.0, 90.0, 180.0])
def test_rotation_about_centre(cm, deg):
    # truth: a turn by delta about the common centre; every corner of an
    # n x n image lies r = (n - 1)/sqrt(2) from it and moves by 2 r sin(delta/2)
    n = 101
    d = math.radians(deg)
    c = (n - 1) / 2.0
    ct, st = math.cos(d), math.sin(d)
    t = (ct, -st, c - ct * c + st * c, st, ct, c - st * c - ct * c)
    r = (n - 1) / math.sqrt(2.0)
    want = 2.0 * r * math.sin(d / 2.0)
    got = cm.cmif_corner_error(best(), (n, n, n, n), t)
    assert abs(got - want) < 1e-9, (got, want)


def test_result_matching_generator_truth_is_zero(cm):
    # the generators' truth and the result convention describe the same map
    rng = np.random.default_rng(5)
    for _ in range(20):
        n = int(rng.integers(20, 600))
        th = float(rng.uniform(0.0, 360.0))
        s = (int(rng.integers(-30, 31)), int(rng.integers(-30, 31)))
        t = synth.truth_a_to_b(th, s, n)
        e = cm.cmif_corner_error(best(0, math.radians(th), s[0], s[1]),
                                 (n, n, n, n), t)
        assert e < 1e-9, e
        # an angle wrong by one degree turns each corner's image about the
        # centre: corner x moves by 2 sin(0.5 deg) |x + chi - c|
        e1 = cm.cmif_corner_error(best(0, math.radians(th + 1.0), s[0], s[1]),
                                  (n, n, n, n), t)
        c = (n - 1) / 2.0
        want = np.mean([2.0 * math.sin(math.radians(0.5)) *
                        math.hypot(x + s[1] - c, y + s[0] - c)
                        for x in (0, n - 1) for y in (0, n - 1)])
        assert abs(e1 - want) < 1e-9 * n, (e1, want)


def test_invalid_arguments(cm):
    with pytest.raises(cm.CmifError):
        cm.cmif_corner_error(best(), (0, 5, 5, 5), IDENT)
