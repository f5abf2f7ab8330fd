"""Hand-worked pins of oracle functions whose earlier pins left plausible mistakes open.

Every expected value here is derived by hand from the definition the paper gives (or the
reading taken where it is silent), written out step by step in plain Python floats, with no
call into the oracle's arithmetic:

- strength of connection (Sec. 4: classical Ruge-Stueben, theta = 0.25) on a 6-node matrix
  with unequal couplings, positive couplings, an exact tie at the threshold and a row whose
  couplings are all positive: catches |a_ij| in place of -a_ij and > in place of >=;
- the off-diagonal scale s of Eq. 5 (Sec. 3.1) on levels with stored zero off-diagonals;
- the GCIN forward (Sec. 3.2, Eqs. 6-10; App. A.1) on a 3-node graph with chosen weights:
  catches a self-loop weight of a_ii instead of 1, ReLU before InstanceNorm, the unbiased
  variance, sum- instead of mean-pooling, a missing max-pooling, and sigmoid before or
  without the LayerNorm;
- the sign of the validation metric (Sec. 3.3, Eq. 13) on a case with a known ordering.
"""
import math

import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import amg, grad
from oracle import gcin as OG


def _sym(n, diag, edges):
    """Symmetric CSR from a diagonal and {(i, j): a_ij} for i < j."""
    rows, cols, vals = list(range(n)), list(range(n)), list(diag)
    for (i, j), a in edges.items():
        rows += [i, j]
        cols += [j, i]
        vals += [a, a]
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A


# ---------------------------------------------------------------------------------------------
# Strength of connection: S_i = { j != i : -a_ij >= theta max_{k != i}(-a_ik) }, theta = 0.25
# ---------------------------------------------------------------------------------------------


def test_strength_hand_worked_six_nodes():
    A = _sym(6, [10.0, 7.0, 7.0, 6.0, 2.0, 2.0], {
        (0, 1): -4.0, (0, 2): -1.0, (0, 3): 2.0, (0, 4): -0.9,
        (1, 2): -2.0, (2, 3): -3.0, (3, 4): 0.5, (3, 5): 1.0,
    })
    # row 0: -a = {1: 4, 2: 1, 3: -2, 4: 0.9}; max 4, threshold 1.0 -> 1 (4 >= 1), 2 (1 >= 1, the
    #        tie is strong), not 3 (positive coupling), not 4 (0.9 < 1)
    # row 1: -a = {0: 4, 2: 2}; max 4, threshold 1 -> both
    # row 2: -a = {0: 1, 1: 2, 3: 3}; max 3, threshold 0.75 -> all three
    # row 3: -a = {0: -2, 2: 3, 4: -0.5, 5: -1}; max 3, threshold 0.75 -> only 2 (with |a_ij|,
    #        0 would be strong too)
    # row 4: -a = {0: 0.9, 3: -0.5}; max 0.9, threshold 0.225 -> only 0 (|a_43| = 0.5 would pass)
    # row 5: -a = {3: -1}; no negative coupling, max <= 0 -> empty
    expect = {0: [1, 2], 1: [0, 2], 2: [0, 1, 3], 3: [2], 4: [0], 5: []}
    S = amg.strength(A, 0.25)
    for i, cols in expect.items():
        assert list(S.indices[S.indptr[i]:S.indptr[i + 1]]) == cols, i


def test_strength_threshold_half_hand_worked():
    """The same matrix at theta = 0.5: row 0 keeps only 1 (1 < 2), row 1 both (2 >= 2), row 2
    keeps 1 and 3 (1 < 1.5), row 4 still only 0."""
    A = _sym(6, [10.0, 7.0, 7.0, 6.0, 2.0, 2.0], {
        (0, 1): -4.0, (0, 2): -1.0, (0, 3): 2.0, (0, 4): -0.9,
        (1, 2): -2.0, (2, 3): -3.0, (3, 4): 0.5, (3, 5): 1.0,
    })
    expect = {0: [1], 1: [0, 2], 2: [1, 3], 3: [2], 4: [0], 5: []}
    S = amg.strength(A, 0.5)
    for i, cols in expect.items():
        assert list(S.indices[S.indptr[i]:S.indptr[i + 1]]) == cols, i


# ---------------------------------------------------------------------------------------------
# Off-diagonal scale of Eq. 5 on levels without a nonzero off-diagonal
# ---------------------------------------------------------------------------------------------


def test_scale_with_stored_zero_offdiagonals_is_one():
    """s = max |offdiag| is undefined when every stored off-diagonal is 0; the reading takes s = 1,
    which makes q_ii = f_d(a_ii)/a_ii and q_ij = 0 (f_o(0) = 0): finite values."""
    A = sp.csr_matrix((np.array([2.0, 0.0, 0.0, 4.0]), np.array([0, 1, 0, 1]), np.array([0, 2, 4])), shape=(2, 2))
    assert A.nnz == 4  # the zeros are stored
    assert amg.offdiag_scale(A) == 1.0
    Q = amg.assemble_smoother(A, [0.5, 0.25, 0.0, 0.3, 0.1], 2)
    # q_00 = (0.5 + 2 * 0.25) / 2 = 0.5; q_11 = (0.5 + 4 * 0.25) / 4 = 0.375; q_01 = q_10 = 0
    assert np.array_equal(Q.data, np.array([0.5, 0.0, 0.0, 0.375]))
    D = sp.csr_matrix((np.array([3.0, 5.0]), np.array([0, 1]), np.array([0, 1, 2])), shape=(2, 2))
    assert amg.offdiag_scale(D) == 1.0
    # one nonzero among stored zeros: s = |a_ij|
    B = sp.csr_matrix((np.array([2.0, -0.5, -0.5, 4.0]), np.array([0, 1, 0, 1]), np.array([0, 2, 4])), shape=(2, 2))
    assert amg.offdiag_scale(B) == 0.5


# ---------------------------------------------------------------------------------------------
# GCIN forward, worked by hand on a 3-node graph
# ---------------------------------------------------------------------------------------------

EPS = 1e-5


def _sigmoid(x):
    return 1.0 / (1.0 + math.exp(-x))


def _hand_params(degree=2):
    """Weights chosen so that every step can be followed on paper (64 channels, 4 layers)."""
    p = {k: np.zeros(s) for k, s in OG.param_shapes(degree)}
    # layer 0: channel 0 <- aggregated a_ii, channel 1 <- aggregated degree
    p["conv0.W"][0, 0] = 1.0
    p["conv0.W"][1, 1] = 1.0
    p["norm0.gamma"][:] = 1.0
    p["norm0.gamma"][0] = 2.0
    p["norm0.beta"][0] = 0.5
    p["norm0.beta"][1] = -0.25
    p["norm0.beta"][2] = 0.3
    p["norm0.beta"][3] = -0.1
    # layer 1: identity weights, unit gains, zero shifts
    p["conv1.W"][:, :] = np.eye(64)
    p["norm1.gamma"][:] = 1.0
    # layers 2, 3: zero gains and shifts -> outputs relu(0) = 0
    # readout of layer 0: out 0 = mean ch0, out 1 = max ch0, out 2 = mean ch1, out 3 = max ch2
    p["readout0.W"][0, 0] = 1.0
    p["readout0.W"][64 + 0, 1] = 1.0
    p["readout0.W"][1, 2] = 1.0
    p["readout0.W"][64 + 2, 3] = 1.0
    # readout of layer 1: out 0 = mean ch0, out 1 = max ch2, bias 0.2 on out 5
    p["readout1.W"][0, 0] = 1.0
    p["readout1.W"][64 + 2, 1] = 1.0
    p["readout1.b"][5] = 0.2
    p["ln.gamma"][:] = 1.0
    p["ln.beta"][0] = 0.1
    p["mlp0.W"][:, :] = np.eye(128)
    p["mlp1.W"][:64, :] = np.eye(64)
    # coefficients: c0 <- t0, c1 <- t1, c2 <- t2, c3 <- t32, c4 <- t33 + 0.01
    p["mlp2.W"][0, 0] = 1.0
    p["mlp2.W"][1, 1] = 1.0
    p["mlp2.W"][2, 2] = 1.0
    p["mlp2.W"][32, 3] = 1.0
    p["mlp2.W"][33, 4] = 1.0
    p["mlp2.b"][4] = 0.01
    return p


def _hand_forward():
    """The forward of _hand_params on A = [[2, -1, 0], [-1, 3, -2], [0, -2, 1]], by hand."""
    # Eq. 6 features [a_ii, deg]: node 0 [2, 1], node 1 [3, 2], node 2 [1, 1].
    # Eq. 8 A_hat = off-diagonal part + unit self-loops: rows [1, -1, 0], [-1, 1, -2], [0, -2, 1].
    # Layer 0 aggregation H = A_hat X:
    #   node 0: [2 - 3, 1 - 2] = [-1, -1]; node 1: [-2 + 3 - 2, -1 + 2 - 2] = [-1, -1];
    #   node 2: [-6 + 1, -4 + 1] = [-5, -3]
    # Theta_0 copies them into channels 0 and 1; the other channels are 0.
    # InstanceNorm (biased variance over the 3 nodes):
    #   ch0 [-1, -1, -5]: mean -7/3, deviations [4/3, 4/3, -8/3], variance (16+16+64)/27 = 32/9
    #   ch1 [-1, -1, -3]: mean -5/3, deviations [2/3, 2/3, -4/3], variance (4+4+16)/27 = 8/9
    #   ch2.. [0, 0, 0]: deviations 0 -> normalised 0
    n0 = [d / math.sqrt(32.0 / 9.0 + EPS) for d in (4 / 3, 4 / 3, -8 / 3)]
    n1 = [d / math.sqrt(8.0 / 9.0 + EPS) for d in (2 / 3, 2 / 3, -4 / 3)]
    # affine then ReLU: ch0 relu(2 n + 0.5), ch1 relu(n - 0.25), ch2 relu(0.3), ch3 relu(-0.1) = 0
    x0 = [max(0.0, 2 * v + 0.5) for v in n0]          # [a, a, 0] since 2 n0[2] + 0.5 < 0
    x1 = [max(0.0, v - 0.25) for v in n1]             # [b, b, 0]
    x2 = [0.3, 0.3, 0.3]
    assert x0[2] == 0.0 and x1[2] == 0.0
    a, b = x0[0], x1[0]
    # readout of layer 0: [mean ch0, max ch0, mean ch1, max ch2]
    r0 = [(2 * a) / 3, a, (2 * b) / 3, 0.3]
    # Layer 1 (identity Theta, zero bias): H = A_hat X^(0)
    #   ch0 [a, a, 0] -> node 0: a - a = 0; node 1: -a + a - 0 = 0; node 2: -2a
    #     mean -2a/3, deviations [2a/3, 2a/3, -4a/3], variance (4+4+16) a^2/27 = 8a^2/9
    #   ch2 [0.3, 0.3, 0.3] -> node 0: 0; node 1: -0.3 + 0.3 - 0.6 = -0.6; node 2: -0.6 + 0.3 = -0.3
    #     mean -0.3, deviations [0.3, -0.3, 0], variance 0.18/3 = 0.06
    m0 = [d / math.sqrt(8 * a * a / 9 + EPS) for d in (2 * a / 3, 2 * a / 3, -4 * a / 3)]
    m2 = [d / math.sqrt(0.06 + EPS) for d in (0.3, -0.3, 0.0)]
    y0 = [max(0.0, v) for v in m0]   # unit gain, zero shift
    y2 = [max(0.0, v) for v in m2]
    r1 = [sum(y0) / 3, max(y2)]
    # concatenation (Eq. 10): z[0:4] = r0, z[32] = r1[0], z[33] = r1[1], z[37] = 0.2, else 0
    z = [0.0] * 128
    z[0:4] = r0
    z[32], z[33], z[37] = r1[0], r1[1], 0.2
    mean = sum(z) / 128
    var = sum((v - mean) ** 2 for v in z) / 128
    zn = [(v - mean) / math.sqrt(var + EPS) for v in z]
    zn[0] += 0.1  # LayerNorm shift on entry 0
    s = [_sigmoid(v) for v in zn]
    # MLP: identity 128 -> 128, first 64 of them, ReLU keeps the positive sigmoid values
    t = s[:64]
    return np.array([t[0], t[1], t[2], t[32], t[33] + 0.01])


def test_gcin_forward_hand_worked_three_nodes():
    A = _sym(3, [2.0, 3.0, 1.0], {(0, 1): -1.0, (1, 2): -2.0})
    got = OG.forward_np(_hand_params(), [A], 2)[0]
    ref = _hand_forward()
    assert np.allclose(got, ref, rtol=0, atol=1e-12), (got, ref)


def test_gcin_forward_hand_worked_values_are_discriminating():
    """The worked example is not degenerate: the five coefficients differ from each other and
    from sigmoid(0) = 0.5, so each of the listed mistakes moves at least one of them."""
    ref = _hand_forward()
    assert len(set(np.round(ref, 6))) == 5
    assert np.all(np.abs(ref - 0.5) > 1e-3)


# ---------------------------------------------------------------------------------------------
# Validation metric (Eq. 13): log10(||r|| / ||r_omega-J||), negative when better than Jacobi
# ---------------------------------------------------------------------------------------------


def test_validation_metric_sign_no_smoothing_is_worse():
    """With every coefficient zero the cycle does no smoothing (Q = 0), so only the coarse-grid
    correction acts: on the 5-point grid it leaves the oscillatory residual untouched, which
    omega-Jacobi damps by at least a factor 3 (its smoothing factor is 1/3 at omega = 2/3).
    Eq. 13 must then be positive, and by at least log10(3)/2 here."""
    A, f = W.poisson_grid_64(3)
    An, fn, sing = amg.normalize(A, f)
    h = amg.setup(An, max_levels=3, singular=sing)
    zero = np.zeros((h.nlevels, 5))
    v = grad.validation_metric(h, zero, 2, fn)
    assert v > 0.5 * math.log10(3.0), v
    # and the metric is the difference of the two losses (one cycle from u = 0)
    jac = np.tile(amg.jacobi_coeffs(), (h.nlevels, 1))
    diff = grad.vcycle_loss(h, zero, 2, fn) - grad.vcycle_loss(h, jac, 2, fn)
    assert abs(v - diff) <= 1e-12
