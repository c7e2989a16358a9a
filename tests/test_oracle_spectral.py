"""Pins of the oracle's transforms and explicit operator (CPU only)."""
import numpy as np
import pytest

from oracle import spectral as sp, stepper
from synthetic import initial_field
from tests import pins


def _rand_box(N, seed, kz=0.7):
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    return b * sp.box_mask(N)[None]


@pytest.mark.parametrize("N", [8, 16])
def test_transforms_match_brute_force_sums(N):
    """Coefficient convention b(x) = sum_k bh e^{ik.x}, both directions."""
    rng = np.random.default_rng(N)
    bh = rng.standard_normal((3, N, N)) + 1j * rng.standard_normal((3, N, N))
    f = sp.to_physical(bh)
    ref = pins.brute_synthesis(bh)
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))
    back = sp.to_spectral(f)
    ref2 = pins.brute_analysis(f)
    assert np.max(np.abs(back - ref2)) <= 1e-14 * np.max(np.abs(ref2))
    assert np.max(np.abs(back - bh)) <= 1e-14 * np.max(np.abs(bh))


def test_box_size_and_wavenumbers():
    assert sp.box_K(32) == 10 and sp.box_K(128) == 42 and sp.box_K(512) == 170
    assert int(sp.box_mask(128).sum()) == 85 * 85
    k = sp.wavenumbers(8)
    assert list(k) == [0, 1, 2, 3, -4, -3, -2, -1]


@pytest.mark.parametrize("flow", ["roberts", "gp"])
@pytest.mark.parametrize("N,t", [(16, 0.0), (16, 1.3), (32, 4.1)])
def test_explicit_term_matches_direct_convolution(flow, N, t):
    bh = _rand_box(N, 7 + N)
    got = sp.explicit_term(bh, flow, 0.57, t)
    ref = pins.direct_explicit(bh, flow, 0.57, t)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_explicit_term_none_is_zero():
    bh = _rand_box(16, 3)
    assert np.all(sp.explicit_term(bh, "none", 1.0, 0.0) == 0)


@pytest.mark.parametrize("N,kz", [(16, 1.0), (32, 2.87)])
def test_curl_form_equals_roberts_component_equations(N, kz):
    """Section 2.1: for solenoidal b the curl form reduces to the b_x and
    b_y equations of the Roberts dynamo."""
    bh = initial_field(N, kz, 11, amp=1.0, kmax=N / 3)
    assert np.max(np.abs(sp.divergence(bh, kz))) < 1e-12
    got = sp.explicit_term(bh, "roberts", kz, 0.0)[:2]
    ref = pins.advective_roberts(bh, kz)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("t", [0.0, 0.9, 2.5])
def test_curl_form_equals_gp_component_equations(t):
    """Section 2.2 (relabelled): same check for the Galloway-Proctor flow."""
    N, kz = 32, 0.57
    bh = initial_field(N, kz, 12, amp=1.0, kmax=N / 3)
    got = sp.explicit_term(bh, "gp", kz, t)[:2]
    ref = pins.advective_gp(bh, kz, t)
    assert np.linalg.norm(got - ref) <= 1e-13 * np.linalg.norm(ref)


def test_a_sign_error_in_the_curl_is_caught():
    """A planted mistake (flipped y-component of the curl) must fail the
    convolution pin: guards that the pin is sensitive."""
    N, kz, t = 16, 0.57, 0.4
    bh = _rand_box(N, 5)
    good = sp.explicit_term(bh, "gp", kz, t)
    bad = good.copy()
    bad[1] = -bad[1]
    ref = pins.direct_explicit(bh, "gp", kz, t)
    assert np.linalg.norm(bad - ref) > 1e-3 * np.linalg.norm(ref)
    assert np.linalg.norm(good - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("flow", ["roberts", "gp"])
def test_divergence_free_is_preserved(flow):
    N, kz = 32, 0.57
    b0 = initial_field(N, kz, 21)
    b = stepper.propagate(b0, flow, 50.0, kz, 0.3, 1e-2, 40)
    k = sp.wavenumbers(N)
    scale = np.max(np.sqrt(k[None, :] ** 2 + k[:, None] ** 2 + kz ** 2)
                   * np.sqrt(np.sum(np.abs(b) ** 2, axis=0)))
    assert np.max(np.abs(sp.divergence(b, kz))) <= 1e-13 * scale


@pytest.mark.parametrize("flow", ["roberts", "gp"])
def test_propagator_is_linear(flow):
    N, kz = 16, 0.57
    a = initial_field(N, kz, 31)
    c = initial_field(N, kz, 32)
    al, be = 0.3 - 1.2j, -2.0 + 0.5j
    f = lambda x: stepper.propagate(x, flow, 20.0, kz, 1.1, 1e-2, 25)
    lhs = f(al * a + be * c)
    rhs = al * f(a) + be * f(c)
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(rhs)
