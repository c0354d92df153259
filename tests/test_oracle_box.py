"""Pins of the box check: the interval it reports is the exact range of the
output over the box (brute force over all vertices), the counter-example
lies in the box and reaches the unsafe interval, and the first violation is
the earliest step."""
import itertools

import numpy as np
import pytest

from oracle import box_check


def _vertices_range(M, roles, zc, r):
    gi = [i for i, x in enumerate(roles) if x == "gen"]
    fi = [i for i, x in enumerate(roles) if x != "gen"]
    vals = []
    for signs in itertools.product((-1.0, 1.0), repeat=len(gi)):
        z = zc + np.array(signs) * r
        vals.append(M[gi] @ z + M[fi].sum())
    return min(vals), max(vals)


@pytest.mark.parametrize("seed", range(6))
def test_range_is_exact_over_box(seed):
    rng = np.random.default_rng(seed)
    S1, o, ng = 7, 3, 5
    roles = ["gen"] * ng + ["center", "affine"]
    basis = rng.normal(size=(S1, o, ng + 2))
    basis[2, 1, 1] = 0.0                      # a zero coefficient
    zc = rng.normal(size=ng); r = rng.uniform(0, 1, size=ng)
    unsafe = np.array([[np.inf, np.inf]] * o)
    res = box_check(basis, roles, zc, r, unsafe)
    for s in range(S1):
        for q in range(o):
            lo, hi = _vertices_range(basis[s, q], roles, zc, r)
            assert abs(res["lo"][s, q] - lo) <= 1e-12 * (1 + abs(lo))
            assert abs(res["hi"][s, q] - hi) <= 1e-12 * (1 + abs(hi))
    assert res["first_step"] == -1


@pytest.mark.parametrize("seed", range(8))
def test_counter_example_is_valid_and_first(seed):
    rng = np.random.default_rng(100 + seed)
    S1, o, ng = 9, 2, 4
    roles = ["gen"] * ng + ["affine"]
    basis = rng.normal(size=(S1, o, ng + 1))
    zc = rng.normal(size=ng); r = rng.uniform(0.1, 1, size=ng)
    probe = box_check(basis, roles, zc, r, np.array([[np.inf, np.inf]] * o))
    # put an unsafe interval that the range at a random (s, q) meets partly
    s0, q0 = int(rng.integers(2, S1)), int(rng.integers(0, o))
    lo, hi = probe["lo"][s0, q0], probe["hi"][s0, q0]
    kind = seed % 3
    if kind == 0:
        U = (lo + 0.7 * (hi - lo), np.inf)          # above the center
    elif kind == 1:
        U = (-np.inf, lo + 0.2 * (hi - lo))         # below the center
    else:
        c = 0.5 * (lo + hi); U = (c - 1e-3, c + 1e-3)
    unsafe = np.array([[np.inf, np.inf]] * o)
    unsafe[q0] = U
    res = box_check(basis, roles, zc, r, unsafe)
    s, q = res["first_step"], res["row"]
    assert s != -1 and (s, q) <= (s0, q0)
    hit = probe["lo"][:, q0] <= U[1]
    hit &= probe["hi"][:, q0] >= U[0]
    assert s == int(np.argmax(hit)) and q == q0
    z = res["z"]
    assert np.all(z >= zc - r - 1e-12) and np.all(z <= zc + r + 1e-12)
    y = basis[s, q, :ng] @ z + basis[s, q, ng]
    assert abs(y - res["y"]) <= 1e-10 * (1 + abs(y))
    assert U[0] - 1e-10 <= y <= U[1] + 1e-10


def test_safe_when_unsafe_interval_empty_of_range():
    basis = np.ones((3, 1, 2))
    res = box_check(basis, ["gen", "affine"], np.array([0.0]), np.array([0.5]),
                    np.array([[2.0, np.inf]]))
    assert res["first_step"] == -1
    res = box_check(basis, ["gen", "affine"], np.array([0.0]), np.array([0.5]),
                    np.array([[1.5, np.inf]]))
    assert res["first_step"] == 0 and abs(res["y"] - 1.5) < 1e-15 and abs(res["z"][0] - 0.5) < 1e-15
