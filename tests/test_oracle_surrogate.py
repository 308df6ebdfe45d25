"""Pins for the oracle of the learned force model: the channel basis
reproduces the gauge force, the auxiliary channel passes a force through,
gauge covariance (with and without the auxiliary field), finite-difference
gradients, bfloat16 rounding and Adam."""
import numpy as np
import pytest

import synth
from oracle import gauge, lattice as L, surrogate as S
from oracle.su3 import to_coords, to_matrix

DIMS = (4, 4, 2, 4)


def _U(kind=0, eps=0.6):
    return synth.random_su3_near_identity(DIMS, eps, synth.make_rng(600, kind))


def test_basis_with_constant_coefficients_is_the_gauge_force():
    """c_j = -beta/3 for every channel gives -(beta/3) Im tr(T_a U sum_j S_j),
    the Wilson gauge force, because the six channels are the six staples."""
    U = _U()
    f, loops = S.features(U, DIMS)
    B = S.basis(loops)
    F = np.einsum("nj,nja->na", np.full((B.shape[0], S.N_CH), -5.4 / 3), B)
    nx, ny, nz, nt = DIMS
    assert np.abs(F.reshape(nt, nz, ny, nx, 4, 8) - gauge.gauge_force(U, DIMS, 5.4)).max() < 1e-12
    # each plaquette appears in the loops of its 4 links (real parts of the traces)
    plaq_sum = gauge.mean_plaquette(U, DIMS) * 3 * 6 * L.volume(DIMS)
    assert abs(f[:, 0:12:2].sum() - 4 * plaq_sum) < 1e-9


def _rotate(Om, F):
    """A force field transformed by the gauge transformation Om (adjoint at x)."""
    return to_coords(np.einsum("...ij,...mjk,...lk->...mil", Om, to_matrix(F), Om.conj()))


def test_auxiliary_channel_alone_reproduces_the_auxiliary_force():
    """With W3 = 0 and b3 = e_6 every link takes c_6 = 1 and nothing else, so
    the model force is the auxiliary field itself; its feature is the cosine
    of the angle with the staple sum, so the field along the staple sum gives 1."""
    U = _U(4)
    rng = synth.make_rng(600, 5)
    params = S.init_params(rng)
    params["W3"][:] = 0.0
    params["b3"][:] = 0.0
    params["b3"][6] = 1.0
    aux = rng.standard_normal((DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 8))
    assert np.abs(S.surrogate_force(params, U, DIMS, aux=aux) - aux).max() < 1e-13
    gforce = gauge.gauge_force(U, DIMS, 3.0)     # -(beta/3) times the staple sum
    f, _ = S.features(U, DIMS, aux=-gforce)
    assert np.abs(f[:, 14] - 1.0).max() < 1e-12
    f0, _ = S.features(U, DIMS)
    assert np.array_equal(f0[:, 14], np.zeros(f0.shape[0]))


@pytest.mark.parametrize("with_aux", [False, True])
def test_model_force_is_gauge_covariant(with_aux):
    U = _U(1)
    rng = synth.make_rng(600, 9)
    params = S.init_params(rng)
    params["W3"] = rng.standard_normal(params["W3"].shape)
    Om = synth.haar_su3(DIMS, rng)[..., 0, :, :]
    Ug = np.empty_like(U)
    for mu in range(4):
        Ug[..., mu, :, :] = np.einsum("...ij,...jk,...lk->...il", Om, U[..., mu, :, :], L.fwd(Om, mu).conj())
    aux = rng.standard_normal((DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 8)) if with_aux else None
    F = S.surrogate_force(params, U, DIMS, aux=aux)
    Fg = S.surrogate_force(params, Ug, DIMS, aux=None if aux is None else _rotate(Om, aux))
    assert np.abs(_rotate(Om, F) - Fg).max() < 1e-10 * np.abs(F).max()


def test_gradients_match_finite_differences():
    U = _U(2)
    rng = synth.make_rng(600, 3)
    params = S.init_params(rng)
    params["W3"] = rng.standard_normal(params["W3"].shape) * 0.3
    params["b1"] = rng.standard_normal(S.HID) * 0.1
    aux = rng.standard_normal((DIMS[3], DIMS[2], DIMS[1], DIMS[0], 4, 8))
    f, loops = S.features(U, DIMS, aux)
    B = S.basis(loops, aux)
    target = rng.standard_normal((f.shape[0], 8))
    _, g = S.loss_and_grad(params, f, B, target)
    h = 1e-6
    for key in params:
        flat = params[key].reshape(-1)
        for idx in rng.choice(flat.size, size=min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = S.loss_and_grad(params, f, B, target)
            flat[idx] = old - h
            lm, _ = S.loss_and_grad(params, f, B, target)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[key].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (key, idx, fd, an)


def test_bf16_rounding():
    vals = np.array([1.0, 3.140625, 0.1, -2.5, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 65504.0])
    exp = np.array([1.0, 3.140625, 0.10009765625, -2.5, 1.0, 1.015625, 65536.0])
    assert np.array_equal(S.bf16(vals), exp)


def test_adam_first_step_closed_form():
    """With bias correction the first Adam step moves every parameter by
    -lr g / (|g| + eps) (m_1 / (1 - b1) = g, v_1 / (1 - b2) = g^2): about lr
    against the gradient's sign for |g| >> eps, and g / (|g| + eps) of it for
    tiny gradients (which places eps outside the square root)."""
    lr, eps = 0.01, 1e-8
    g = np.array([0.3, -2.0, 1e-9, -3e-9, 0.0, 5e3])
    params = {"w": np.zeros_like(g)}
    S.adam_step(params, {"w": g}, {}, lr=lr)
    exp = -lr * g / (np.abs(g) + eps)
    assert np.allclose(params["w"], exp, rtol=1e-12, atol=0.0)
    # a step without bias correction would be (1-b1)/sqrt(1-b2) = 3.16 times longer
    assert abs(params["w"][1] - lr) < 1e-9


def test_adam_second_step_by_hand():
    """Two steps with gradients g1 then g2, written out:
    m_2 / (1 - b1^2) = (b1 g1 + g2) / (1 + b1),  v_2 / (1 - b2^2) = (b2 g1^2 + g2^2) / (1 + b2),
    step_2 = -lr (b1 g1 + g2) / (1 + b1) / (sqrt((b2 g1^2 + g2^2) / (1 + b2)) + eps)."""
    lr, b1, b2, eps = 0.05, 0.9, 0.999, 1e-8
    g1 = np.array([1.0, 0.5, -2.0, 1.0])
    g2 = np.array([0.0, 0.5, 3.0, -1.0])
    params = {"w": np.array([0.1, 0.2, 0.3, 0.4])}
    state = {}
    S.adam_step(params, {"w": g1}, state, lr=lr)
    w1 = params["w"].copy()
    S.adam_step(params, {"w": g2}, state, lr=lr)
    step2 = -lr * ((b1 * g1 + g2) / (1 + b1)) / (np.sqrt((b2 * g1 ** 2 + g2 ** 2) / (1 + b2)) + eps)
    assert np.allclose(params["w"] - w1, step2, rtol=1e-12, atol=1e-15)
    # first entry worked out by hand (g1 = 1, g2 = 0; eps changes it by 5e-10)
    assert abs((params["w"][0] - w1[0]) - (-lr * (0.9 / 1.9) / np.sqrt(0.999 / 1.999))) < 1e-9
    # an unchanged gradient keeps the step at lr (eps changes it by 1e-9)
    assert abs((params["w"][1] - w1[1]) + lr) < 2e-9


def test_adam_minimises_a_quadratic():
    params = {"w": np.array([3.0, -2.0])}
    state = {}
    for _ in range(2000):
        S.adam_step(params, {"w": 2 * params["w"]}, state, lr=0.05)
    assert np.abs(params["w"]).max() < 1e-3
