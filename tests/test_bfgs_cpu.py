"""The BFGS update of the quasi-Newton trust region (host arithmetic in the C-ABI library, no
device), pinned by the properties that define it (Nocedal & Wright 2006, Sec. 6.1):

* the secant condition B+ s = y and its inverse form H+ y = s;
* symmetry, and positive definiteness kept whenever s^T y > 0;
* H+ is the inverse of B+;
* the change is rank two and leaves B v unchanged for every v with s^T B v = 0 and y^T v = 0;
* the first-update scaling resets B to (y^T y / y^T s) I before updating.
"""
import numpy as np
import pytest

from paper_2505_00529_amd import qoc


def _spd(rng, r):
    a = rng.normal(size=(r, r))
    return a @ a.T + r * np.eye(r)


def _pair(rng, r, b):
    while True:
        s = rng.normal(size=r)
        y = b @ s + 0.3 * rng.normal(size=r)
        if s @ y > 0.1 * np.linalg.norm(s) * np.linalg.norm(y):
            return s, y


@pytest.mark.parametrize("r", [1, 2, 5, 17])
def test_secant_symmetry_inverse_and_definiteness(r):
    rng = np.random.default_rng(40 + r)
    b = _spd(rng, r)
    h = np.linalg.inv(b)
    b0 = b.copy()
    for _ in range(6):
        s, y = _pair(rng, r, b0)
        qoc.bfgs_update(b, h, s, y)
        scale = np.linalg.norm(b)
        assert np.linalg.norm(b @ s - y) < 1e-12 * scale * np.linalg.norm(s)
        assert np.linalg.norm(h @ y - s) < 1e-12 * np.linalg.norm(h) * np.linalg.norm(y)
        assert np.array_equal(b, b.T) or np.abs(b - b.T).max() < 1e-14 * scale
        assert np.abs(h - h.T).max() < 1e-14 * np.linalg.norm(h)
        assert np.linalg.norm(h @ b - np.eye(r)) < 1e-10 * np.linalg.cond(b)
        assert np.linalg.eigvalsh(b).min() > 0


def test_rank_two_change_fixes_the_complement():
    rng = np.random.default_rng(7)
    r = 9
    b = _spd(rng, r)
    h = np.linalg.inv(b)
    s, y = _pair(rng, r, b)
    b_old = b.copy()
    qoc.bfgs_update(b, h, s, y)
    sv = np.linalg.svd(b - b_old, compute_uv=False)
    assert sv[2] < 1e-12 * sv[0]
    # complement: vectors orthogonal to B s and to y
    q, _ = np.linalg.qr(np.column_stack([b_old @ s, y, rng.normal(size=(r, r - 2))]))
    comp = q[:, 2:]
    assert np.abs(comp.T @ (b_old @ s)).max() < 1e-12 * np.linalg.norm(b_old @ s)
    assert np.linalg.norm(b @ comp - b_old @ comp) < 1e-12 * np.linalg.norm(b_old)


def test_first_update_rescales_to_curvature_estimate():
    rng = np.random.default_rng(3)
    r = 6
    b = np.eye(r) * 123.0          # overwritten by the reset
    h = np.eye(r) / 123.0
    s, y = _pair(rng, r, _spd(rng, r))
    qoc.bfgs_update(b, h, s, y, rescale=True)
    sc = (y @ y) / (s @ y)
    # the same update applied by hand to the reset matrix sc I: only s, B s = sc s and y enter
    b_ref = sc * np.eye(r) - sc * np.outer(s, s) / (s @ s) + np.outer(y, y) / (y @ s)
    assert np.linalg.norm(b - b_ref) < 1e-13 * np.linalg.norm(b_ref)
    assert np.linalg.norm(b @ s - y) < 1e-12 * np.linalg.norm(y)
    assert np.linalg.norm(h @ b - np.eye(r)) < 1e-12


def test_nonpositive_curvature_is_rejected_and_leaves_inputs():
    r = 3
    b = np.eye(r)
    h = np.eye(r)
    s = np.array([1.0, 0.0, 0.0])
    for y in (np.array([-1.0, 2.0, 0.0]), np.array([0.0, 1.0, 0.0])):
        with pytest.raises(qoc.QocError):
            qoc.bfgs_update(b, h, s, y)
        assert np.array_equal(b, np.eye(r)) and np.array_equal(h, np.eye(r))
    with pytest.raises(ValueError):
        qoc.bfgs_update(np.eye(2), np.eye(3), s, s)
