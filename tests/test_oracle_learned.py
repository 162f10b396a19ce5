"""Pins of the learned-rank oracle: the published Philox4x32-10 answers, the
Box-Muller transform, the feature definition on cases with known answers,
backpropagation against central differences, and the training pairs."""
import numpy as np
import pytest

from oracle import learned
from oracle.hsolver import factor
from oracle.tree import build_tree
from synth import laplace2d, lognormal_field, slab_scalar


def test_philox_known_answers():
    # known-answer vectors of Philox4x32-10 from the Random123 distribution
    cases = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, want in cases:
        got = learned.philox4x32_10(np.array(ctr, np.uint64), np.array(key, np.uint64))
        assert [int(x) for x in got] == want


def test_box_muller():
    # u0 chosen so that -2 ln a = 1 exactly up to the word grid: radius ~ 1
    a = np.exp(-0.5)
    u0 = round(a * 2 ** 32 - 0.5)
    g0, g1 = learned.box_muller(u0, 0)
    r = np.hypot(g0, g1)
    assert abs(r - 1.0) < 1e-9 and g0 > 0.999999 and abs(g1) < 1e-8
    # moments of many draws
    w = learned.philox4x32_10(np.stack([np.arange(40000, dtype=np.uint64)] + [np.zeros(40000, np.uint64)] * 3,
                                       -1), np.array([7, 0], np.uint64))
    z = np.concatenate(learned.box_muller(w[:, 0], w[:, 1]))
    assert abs(z.mean()) < 0.02 and abs(z.var() - 1.0) < 0.02


def _blocks_two(Asy, m=3, n=4, dy=2.0, ds=1.0):
    blocks = {(0, 0): np.eye(m) * ds, (1, 1): np.eye(n) * dy, (0, 1): Asy, (1, 0): Asy.T}
    return blocks, [m, n], [[1], [0]]


def test_features_known_cases():
    rng = np.random.default_rng(0)
    # zero coupling: zero norm and zero singular values; two linked clusters:
    # no far field, cluster 0 first (colour 0), cluster 1 after its neighbour
    F = learned.level_features(0, *_blocks_two(np.zeros((3, 4))), 1e-2)
    assert F[0, 2] < -299 and np.all(F[0, 3:11] == 0)
    assert F[0, 0] == 2.0 and F[0, 1] == 0.0 and F[0, 11] == 0.0
    assert F[1, 0] == np.log2(5.0) and F[1, 11] == 1.0
    # rank-one coupling: one nonzero sketch singular value (the Gram route
    # leaves the others at about sqrt(eps) of the first)
    u, v = rng.standard_normal(3), rng.standard_normal(4)
    F = learned.level_features(0, *_blocks_two(np.outer(u, v)), 1e-2)
    assert F[0, 3] > 0.1 and np.all(F[0, 4:11] < 1e-6 * F[0, 3])
    # Jacobi scaling: ||B||_F of a coupling between unit and 2*I blocks
    A = rng.standard_normal((3, 4))
    F = learned.level_features(0, *_blocks_two(A), 1e-2)
    assert np.isclose(10 ** F[0, 2], np.linalg.norm(A) / np.sqrt(2.0), rtol=1e-12)
    # scaling the whole matrix leaves every feature unchanged
    b2, sz, g = _blocks_two(A)
    F2 = learned.level_features(0, {k: 5.0 * v for k, v in b2.items()}, sz, g, 1e-2)
    assert np.allclose(F, F2, rtol=1e-12, atol=1e-6)  # sqrt(eps) noise of null directions
    # the squared sketch singular values sum to ||B Omega||_F^2
    om = learned.omega(0, 1, 4)
    B = A / np.sqrt(2.0)
    sig = F[0, 3:11] * 10 ** F[0, 2]
    assert np.isclose(np.sum(sig ** 2), np.linalg.norm(B @ om) ** 2, rtol=1e-10)


def test_symbolic_far_field_path():
    # path 0-1-2-3: colours 0,1,2,0 (distance 2), order 0,3,1,2.  Eliminating
    # 0 links nothing new (one neighbour); 3 likewise; 1 (neighbours 0, 2)
    # links 0-2, so 2 then has far field {0}; 1 has none.
    sizes = [2, 3, 5, 7]
    graph = [[1], [0, 2], [1, 3], [2]]
    b, e = learned.symbolic_far_field(graph, sizes)
    assert b.tolist() == [0, 0, 2, 0]
    assert e.tolist() == [0.0, 0.5, 1.0, 0.0]


def _params(seed=0):
    rng = np.random.default_rng(seed)
    d = {"mu": rng.standard_normal(12), "isd": rng.uniform(0.5, 2.0, 12),
         "W1": rng.standard_normal((64, 12)) * 0.3, "b1": rng.standard_normal(64) * 0.1,
         "W2": rng.standard_normal((64, 64)) * 0.15, "b2": rng.standard_normal(64) * 0.1,
         "w3": rng.standard_normal(64) * 0.2, "b3": np.array([0.3])}
    return learned.pack(d)


def test_mlp_backprop_matches_central_differences():
    rng = np.random.default_rng(1)
    p = _params()
    X = rng.standard_normal((20, 12))
    t = rng.uniform(0, 10, 20)
    loss, g = learned.mlp_loss_grad(p, X, t)
    assert g[:24].tolist() == [0.0] * 24  # mu, isd are not trained
    h = 1e-6
    idx = np.concatenate([np.arange(24, 24 + 768, 37), np.arange(24 + 768, learned.NPARAMS, 29),
                          [learned.NPARAMS - 1]])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        fd = (learned.mlp_loss_grad(p + e, X, t)[0] - learned.mlp_loss_grad(p - e, X, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])
    assert learned.NPARAMS == 24 + 768 + 64 + 4096 + 64 + 64 + 1


def test_rank_pairs_follow_the_factor():
    pr = slab_scalar(12, 10, 4, 1e3, lognormal_field((10, 12, 4), seed=3))
    X, k, lv = learned.rank_pairs(pr, 24, 1e-2)
    T = build_tree(pr.grid, 24)
    F = factor(pr.rowptr, pr.col, pr.val, T, 1e-2)
    assert k.tolist() == [float(r) for rec in F.levels for r in rec.ranks]
    assert X.shape == (len(k), 12) and np.isfinite(X).all()
    assert lv.max() == len(F.levels) - 1
