"""Pins for the learned-FSAI oracle: bfloat16 rounding, features, the loss and
every gradient (against dense algebra, hand values and finite differences),
Adam's first step, and the classic FSAI reference."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import oracle
from oracle import fsai
from paper_2608_09647_amd import inputs as I


def test_bf16_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, -3.5e-38]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(fsai.bf16(x), ref)
    assert fsai.bf16(1.00390625) == 1.0          # halfway: ties to even mantissa 0
    assert fsai.bf16(1.01171875) == 1.015625     # halfway: ties to even mantissa 2


def test_param_count_and_packing():
    assert fsai.N_PARAMS == 12 * 64 + 64 + 64 * 64 + 64 + 64 * 5 + 5 == 5317
    th = np.arange(fsai.N_PARAMS, dtype=float)
    assert np.array_equal(fsai.pack(fsai.unpack(th)), th)
    p = fsai.unpack(th)
    assert p["W1"][1, 0] == 12 and p["b3"][-1] == 5316


def test_features_by_hand():
    k = np.array([[1.0, 4.0, 2.0], [8.0, 1.0, 1.0], [2.0, 2.0, 16.0]])
    A = I.diffusion2d(k)
    F = fsai.features(A)
    S = A.scipy().toarray()
    d = np.diag(S)
    # cell (ix=1, iy=1) = row 4 has all four neighbours
    i = 4
    for s, j in enumerate((3, 5, 1, 7)):           # W, E, S, N
        assert F[i, s] == pytest.approx(S[i, j] / np.sqrt(d[i] * d[j]), rel=1e-15)
        assert F[i, 4 + s] == pytest.approx(np.log(d[j] / d[i]), rel=1e-15)
        assert F[i, 8 + s] == 0.0
    # corner (0, 0) = row 0 has no W and no S
    assert list(F[0, 8:]) == [1.0, 0.0, 1.0, 0.0]
    assert F[0, 0] == 0.0 and F[0, 2] == 0.0 and F[0, 4] == 0.0
    assert np.all(np.abs(F[:, :4]) <= 1.0)          # diagonally dominant: |a_ij| <= sqrt(d_i d_j)


def test_slot_index_rejects_non_stencil():
    # row 3 has two entries left of column 2: both would be its S slot
    A = oracle_dense_csr(np.array([[4.0, 0, 0, 1], [0, 4, 0, 1], [0, 0, 4, 0], [1, 1, 0, 4]]))
    with pytest.raises(ValueError):
        fsai.slot_index(A)


def oracle_dense_csr(M):
    S = sp.csr_matrix(M)
    S.sort_indices()
    return I.CSR(M.shape[0], S.indptr.astype(np.int32), S.indices.astype(np.int32), S.data)


def random_outputs(n, seed):
    return np.random.default_rng(seed).standard_normal((n, 5)) * 0.5


def test_loss_matches_dense_formula():
    A = I.diffusion2d(I.log_normal_field(8, 8, [2, 0]))
    o = random_outputs(A.n, 1)
    Gt = fsai.g_tilde(A, o)
    Ahat, d = fsai.scaled_operator(A)
    rows = np.array([0, 5, 17, 40, 63])
    L, dG = fsai.loss_and_grad(Gt, Ahat, rows)
    Gd, Ad = Gt.toarray(), Ahat.toarray()
    E = (Gd @ Ad @ Gd.T - np.eye(A.n))[rows]
    assert L == pytest.approx(np.sum(E * E) / rows.size, rel=1e-13)
    # G = G~ D^-1/2 gives the same product with the unscaled operator
    G = fsai.g_unscaled(Gt, d).toarray()
    assert np.allclose(G @ A.scipy().toarray() @ G.T, Gd @ Ad @ Gd.T, rtol=1e-12, atol=1e-12)
    # the slots: diagonal = softplus(o_C) + 1e-3, W = o_W, S = o_S, nothing above the diagonal
    assert np.allclose(np.diag(Gd), np.logaddexp(0, o[:, 0]) + 1e-3)
    assert Gd[9, 8] == o[9, 1] and Gd[9, 1] == o[9, 3] and np.all(np.triu(Gd, 1) == 0)


def test_loss_is_zero_for_the_exact_factor_of_a_diagonal():
    n = 6
    A = oracle_dense_csr(np.diag([2.0, 3.0, 5.0, 7.0, 11.0, 13.0]))
    o = np.zeros((n, 5))
    o[:, 0] = np.log(np.expm1(1.0 - 1e-3))            # softplus^-1(1 - 1e-3): G~ = I
    Gt = fsai.g_tilde(A, o)
    Ahat, _ = fsai.scaled_operator(A)
    L, dG = fsai.loss_and_grad(Gt, Ahat, np.arange(n))
    assert L < 1e-28 and np.abs(dG.data).max() < 1e-13


def test_loss_gradient_matches_finite_differences():
    A = I.diffusion2d(I.log_normal_field(7, 6, [3, 0]))
    o = random_outputs(A.n, 2)
    Gt = fsai.g_tilde(A, o)
    Ahat, _ = fsai.scaled_operator(A)
    rows = np.array([1, 8, 20, 33, 41])
    L, dG = fsai.loss_and_grad(Gt, Ahat, rows)
    h = 1e-6
    for k in np.random.default_rng(3).choice(Gt.nnz, 25, replace=False):
        Gp, Gm = Gt.copy(), Gt.copy()
        Gp.data[k] += h
        Gm.data[k] -= h
        fd = (fsai.loss_and_grad(Gp, Ahat, rows)[0] - fsai.loss_and_grad(Gm, Ahat, rows)[0]) / (2 * h)
        assert abs(fd - dG.data[k]) <= 1e-6 * max(1.0, abs(fd))


def test_output_gradient_matches_finite_differences():
    A = I.diffusion2d(I.log_normal_field(6, 6, [4, 0]))
    o = random_outputs(A.n, 5)
    Ahat, _ = fsai.scaled_operator(A)
    rows = np.arange(0, A.n, 3)
    _, dG = fsai.loss_and_grad(fsai.g_tilde(A, o), Ahat, rows)
    dO = fsai.grad_outputs(A, o, dG)
    assert np.all(dO[:, 2] == 0) and np.all(dO[:, 4] == 0)      # E and N have no slot
    h = 1e-6
    for i, s in [(0, 0), (7, 0), (7, 1), (14, 3), (35, 1), (35, 3), (20, 0)]:
        op, om = o.copy(), o.copy()
        op[i, s] += h
        om[i, s] -= h
        fd = (fsai.loss_and_grad(fsai.g_tilde(A, op), Ahat, rows)[0]
              - fsai.loss_and_grad(fsai.g_tilde(A, om), Ahat, rows)[0]) / (2 * h)
        assert abs(fd - dO[i, s]) <= 1e-6 * max(1.0, abs(fd))


def test_mlp_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    th = fsai.glorot_init(rng) + 0.01 * rng.standard_normal(fsai.N_PARAMS)
    F = rng.standard_normal((40, 12))
    dO = rng.standard_normal((40, 5))
    g = fsai.mlp_backward(th, F, dO, round_bf16=False)
    f = lambda t: float(np.sum(dO * fsai.mlp_forward(t, F, round_bf16=False)[0]))
    h = 1e-6
    for k in rng.choice(fsai.N_PARAMS, 60, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd))


def test_mlp_forward_plain_formula_and_rounding_points():
    rng = np.random.default_rng(7)
    th = fsai.glorot_init(rng)
    F = rng.standard_normal((10, 12))
    p = fsai.unpack(th)
    ref = np.maximum(np.maximum(F @ p["W1"].T + p["b1"], 0) @ p["W2"].T + p["b2"], 0) @ p["W3"].T + p["b3"]
    o, _ = fsai.mlp_forward(th, F, round_bf16=False)
    assert np.allclose(o, ref, rtol=1e-13, atol=1e-13)
    ob, c = fsai.mlp_forward(th, F, round_bf16=True)
    assert np.array_equal(c["h1"], fsai.bf16(c["h1"])) and np.array_equal(c["f"], fsai.bf16(F))
    assert np.max(np.abs(ob - o)) <= 0.05 * np.max(np.abs(o))


def test_whole_chain_gradient_matches_finite_differences():
    A = I.diffusion2d(I.log_normal_field(5, 5, [5, 0]))
    rng = np.random.default_rng(8)
    th = fsai.glorot_init(rng)
    rows = np.array([0, 6, 12, 18, 24])
    L, g = fsai.network_loss(th, A, rows, round_bf16=False)
    h = 1e-6
    for k in rng.choice(fsai.N_PARAMS, 40, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (fsai.network_loss(tp, A, rows, False)[0] - fsai.network_loss(tm, A, rows, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd))


def test_multi_system_loss_weights_and_gradient():
    """The loss over several systems is the mean over all their sampled rows:
    with unequal row counts its finite differences match the gradient; one
    system reduces to network_loss bit for bit; a system listed twice with
    the same rows gives the single system's loss and gradient (weights 1/2)."""
    systems = [I.diffusion2d(I.log_normal_field(5, 5, [5, 0])),
               I.diffusion2d(I.log_normal_field(6, 4, [6, 0]))]
    rows = [np.array([0, 6, 12, 18, 24]), np.array([1, 9, 22])]
    rng = np.random.default_rng(9)
    th = fsai.glorot_init(rng)
    L, g = fsai.network_loss_multi(th, systems, rows, round_bf16=False)
    Ls = [fsai.network_loss(th, A, r, round_bf16=False)[0] for A, r in zip(systems, rows)]
    assert abs(L - (5 * Ls[0] + 3 * Ls[1]) / 8) <= 1e-14 * L
    h = 1e-6
    for k in rng.choice(fsai.N_PARAMS, 30, replace=False):
        tp, tm = th.copy(), th.copy()
        tp[k] += h
        tm[k] -= h
        fd = (fsai.network_loss_multi(tp, systems, rows, False)[0]
              - fsai.network_loss_multi(tm, systems, rows, False)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd))
    for rb in (False, True):
        L1, g1 = fsai.network_loss(th, systems[0], rows[0], rb)
        Lm, gm = fsai.network_loss_multi(th, systems[:1], rows[:1], rb)
        assert Lm == L1 and np.array_equal(gm, g1)
        L2, g2 = fsai.network_loss_multi(th, [systems[0]] * 2, [rows[0]] * 2, rb)
        assert abs(L2 - L1) <= 1e-15 * L1 and np.allclose(g2, g1, rtol=1e-13, atol=1e-16)


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-12, 0.0])
    th, m, v = fsai.adam_step(np.zeros(4), np.zeros(4), np.zeros(4), g, t=1, lr=1e-3)
    # m_hat = g, v_hat = g^2: the step is lr * g / (|g| + eps)
    assert np.allclose(th, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)


def _adam_bias_slip(theta, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Planted slip: bias correction with beta^1 instead of beta^t."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    return theta - lr * (m / (1 - beta1)) / (np.sqrt(v / (1 - beta2)) + eps), m, v


def _adam_constant_gradient_ok(step):
    """With the same gradient g at every step, the bias-corrected moments are
    exactly g and g^2 at every t (m_t = (1 - beta1^t) g, v_t = (1 - beta2^t)
    g^2), so step t moves theta by -lr g / (|g| + eps): after t steps theta
    = theta_0 - t lr g / (|g| + eps)."""
    g = np.array([0.5, -2.0, 3e-3, 1e-12, 0.0])
    th0 = np.array([0.1, -0.2, 0.3, 0.0, 1.0])
    lr = 1e-3
    th, m, v = th0.copy(), np.zeros(5), np.zeros(5)
    ok = True
    for t in range(1, 6):
        th, m, v = step(th, m, v, g, t, lr=lr)
        want = th0 - t * lr * g / (np.abs(g) + 1e-8)
        ok &= bool(np.allclose(th, want, rtol=0, atol=1e-12 * t))
        ok &= bool(np.allclose(m, (1 - 0.9 ** t) * g, rtol=1e-13, atol=0))
        ok &= bool(np.allclose(v, (1 - 0.999 ** t) * g * g, rtol=1e-12, atol=0))
    return ok


def test_adam_constant_gradient_closed_form_steps_1_to_5():
    assert _adam_constant_gradient_ok(fsai.adam_step)
    assert not _adam_constant_gradient_ok(_adam_bias_slip)


def test_classic_fsai_unit_diagonal_and_gain():
    p = I.diffusion_problem(24, seed=11)
    G = fsai.classic_fsai(p.A)
    S = p.A.scipy()
    M = (G @ S @ G.T).toarray()
    assert np.allclose(np.diag(M), 1.0, rtol=1e-12)
    assert np.all(sp.triu(G, 1).toarray() == 0)
    Gc = I.CSR(p.A.n, *fsai.csr_parts(G))
    Gtc = I.CSR(p.A.n, *fsai.csr_parts(G.T.tocsr()))
    plain = oracle.cg(p.A, p.b, tol=1e-10, maxit=20000)
    pc = oracle.pcg(p.A, Gc, Gtc, p.b, tol=1e-10, maxit=20000)
    assert pc["status"] == oracle.OK and pc["iterations"] < plain["iterations"] / 2
