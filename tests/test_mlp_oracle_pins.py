"""Pins of the FP64 surrogate-network oracle (oracle/mlp.py)."""
import numpy as np

import workloads
from oracle import mlp


def test_parameter_count():
    assert mlp.N_PARAMS == 34052
    assert workloads.mlp_init().shape == (34052,)


def test_silu_closed_forms():
    assert mlp.silu(0.0) == 0.0 and mlp.dsilu(0.0) == 0.5
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.abs(fd - mlp.dsilu(z)).max() < 1e-9
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)))


def test_zero_weights_give_output_bias():
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unflatten(theta)
    p["b4"][:] = [1.5, -2.0, 0.25, 3.0]
    p["b1"][:] = 0.7  # hidden biases do not reach the output through zero W4
    y, _ = mlp.forward(mlp.flatten(p), np.random.default_rng(0).normal(size=(5, 3)))
    assert np.array_equal(y, np.tile([1.5, -2.0, 0.25, 3.0], (5, 1)))


def test_single_hidden_path_closed_form():
    # One path x0 -> unit 0 of every layer -> output 0: y = w4 silu(w3 silu(w2 silu(w1 x0)))
    theta = np.zeros(mlp.N_PARAMS)
    p = mlp.unflatten(theta)
    p["W1"][0, 0], p["W2"][0, 0], p["W3"][0, 0], p["W4"][0, 0] = 0.9, -1.3, 0.7, 2.0
    x = np.array([[0.4, 5.0, -3.0]])
    y, _ = mlp.forward(mlp.flatten(p), x)
    s = mlp.silu
    assert np.isclose(y[0, 0], 2.0 * s(0.7 * s(-1.3 * s(0.9 * 0.4))), rtol=1e-15)
    assert np.all(y[0, 1:] == 0.0)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(3)
    theta = workloads.mlp_init(5)
    x = rng.uniform(0, 1, size=(16, 3))
    t = rng.normal(size=(16, 4))
    w = np.array([1.0, 0.5, 0.5, 0.5])
    _, g = mlp.loss_grad(theta, x, t, w)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    idx = np.concatenate([idx, [0, 383, 384, 511, 34051, 34047, 33536]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tp[i] += h
        tm = theta.copy()
        tm[i] -= h
        fd = (mlp.loss_grad(tp, x, t, w)[0] - mlp.loss_grad(tm, x, t, w)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-3, abs(g[i])) + 1e-10, (i, fd, g[i])


def test_adam_first_step_closed_form():
    # after one step m_hat = g and v_hat = g^2: the update is -lr g/(|g| + eps)
    rng = np.random.default_rng(4)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    th1, m, v = mlp.adam_step(theta, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    assert np.allclose(th1, theta - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=1e-16)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    assert mlp.round_bf16(np.array([one]))[0] == 1.0
    assert mlp.round_bf16(np.array([1 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert mlp.round_bf16(np.array([1 + 3 * 2.0 ** -8]))[0] == 1 + 2.0 ** -6  # tie -> even
    assert mlp.round_bf16(np.array([1 + 2.0 ** -8 + 2.0 ** -20]))[0] == 1 + 2.0 ** -7
    assert mlp.round_bf16(np.array([-3.140625]))[0] == -3.140625


# ------------------------------------ the learned correction, applied ----

def _bias_only(b4):
    p = mlp.unflatten(np.zeros(mlp.N_PARAMS))
    p["b4"][:] = b4
    return mlp.flatten(p)


def test_application_of_a_constant_network_closed_form():
    # A network with only its output bias b outputs b everywhere, so the
    # kernel it stands for is psi(u) = b0 - (2 pi/3)|u|^2 + psi0 with
    # d psi/d r_a = sign(r_a) (b_a - (4 pi/3)|r_a|): the unfold by the sign
    # of each offset and the background term are checked term by term.
    b = np.array([0.3, 0.7, -0.2, 0.05])
    L, psi0, M = 2.0, 21.94, 0.8
    X = np.array([[0.9, 1.1, 1.0]])
    rng = np.random.default_rng(41)
    x = rng.uniform(0, L, size=(40, 3))
    x[0] = [0.9, 1.5, 0.6]  # one offset with two negative components
    acc, pot = mlp.surrogate_correction(_bias_only(b), x, np.array([M]), X, L, psi0)
    r = (x - X[0]) / L
    u = np.abs(r).astype(np.float32).astype(np.float64)
    sgn = np.where(r < 0, -1.0, 1.0)
    psi = b[0] - 2 * np.pi / 3 * (u ** 2).sum(1) + psi0
    for i in range(len(x)):
        assert np.isclose(pot[i], M * psi[i] / L, rtol=1e-14)
        for a in range(3):
            g = sgn[i, a] * (b[1 + a] - 4 * np.pi / 3 * u[i, a])
            assert np.isclose(acc[i, a], -M * g / L ** 2, rtol=1e-13, atol=1e-15)


def test_application_background_term_is_the_same_for_any_cell_split():
    # With a zero network only the quadratic background term remains; its
    # field is linear in the offset, so the sum over cells that split the
    # mass equals the root's alone: sum_c M_c (x - X_c) = M (x - X) for
    # masses and centres of mass of a partition.  This pins the top-cell
    # selection (it must partition the mass, each cell at its own centre).
    import oracle
    ps = workloads.perturbed_lattice(8, 0.25, seed=42)
    t = oracle.build_tree(ps.pos, ps.mass, ps.box_L, 16)
    theta = _bias_only(np.zeros(4))
    x = ps.pos[:64] * 0.5 + 0.25  # offsets stay inside (-1, 1)^3, no folding across 0
    ref_a, ref_p = None, None
    for k in (1, 8, 64):
        cells = mlp.top_cells(t.child, k)
        assert len(set(cells)) == len(cells)
        # a partition: the cells' particle ranges tile [0, n)
        rng_ = sorted((t.cell_first[c], t.cell_count[c]) for c in cells)
        assert rng_[0][0] == 0 and sum(c for _, c in rng_) == ps.n
        assert all(rng_[i][0] + rng_[i][1] == rng_[i + 1][0] for i in range(len(rng_) - 1))
        a, p = mlp.surrogate_correction(theta, x, t.mom[cells, 0], t.com[cells], 1.0, 0.0)
        if k == 1:
            ref_a, ref_p = a, p
            continue
        # (each offset is rounded to float as the network's input: ~6e-8)
        assert np.allclose(a, ref_a, rtol=0, atol=1e-6)
        # the potential's quadratic term differs by the spread of the cells
        # about the root: sum_c M_c |x - X_c|^2 = M |x - X|^2 + sum_c M_c |X_c - X|^2
        spread = (t.mom[cells, 0] * ((t.com[cells] - t.com[0]) ** 2).sum(1)).sum()
        assert np.allclose(p, ref_p - 2 * np.pi / 3 * spread, rtol=0, atol=1e-6)


def test_application_scales_with_box_side():
    theta = workloads.mlp_init(43)
    rng = np.random.default_rng(44)
    x = rng.uniform(0, 1, size=(30, 3))
    X = np.array([[0.5, 0.45, 0.55], [0.2, 0.8, 0.3]])
    M = np.array([0.6, 0.4])
    a1, p1 = mlp.surrogate_correction(theta, x, M, X, 1.0, 21.94)
    for L in (0.5, 4.0):  # powers of two: the offsets scale without rounding
        aL, pL = mlp.surrogate_correction(theta, x * L, M, X * L, L, 21.94)
        assert np.allclose(aL * L * L, a1, rtol=1e-12, atol=1e-14)
        assert np.allclose(pL * L, p1, rtol=1e-12)
