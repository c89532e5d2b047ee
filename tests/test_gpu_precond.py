"""GPU parity of the learned coarse correction against the oracle (oracle/coarse.py,
oracle/mlp.py, oracle/precond.py): pair geometry, low-mode restriction/prolongation,
MLP loss and gradients (float32 kernels vs float64 oracle, 1e-3), the preconditioner
application, and the gain of the trained network over M0."""
import os

import numpy as np
import pytest

from oracle import coarse, mlp
from oracle.grid import Geometry
from oracle.operators import Operators
from oracle.precond import m0_resistance
from tests.gpu_common import assert_close, small_cluster

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bie():
    from paper_1707_06551_amd import bie
    return bie


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def oracle_frames(dirs):
    out = np.zeros((len(dirs), 34))
    for e, d in enumerate(dirs):
        Q = coarse.pair_frame(d)
        out[e, :9] = Q.reshape(-1)
        out[e, 9:] = coarse.rot25(Q)[10:15, 10:15].reshape(-1)
    return out


@pytest.fixture(scope="module")
def cluster():
    c = small_cluster(10, 7.0, 0.05, 21)
    p = 5
    B = _bie()
    s = B.Spheres(c, p, near_gap=1.0)
    g = Geometry(c, p, near_gap=1.0)
    yield c, p, s, g
    s.close()


def test_pair_geometry_matches_oracle(cluster):
    c, p, s, g = cluster
    pi, pj, feats, frames = s.pair_geometry()
    pairs, f_o, dirs = coarse.pair_features(c, g.near, 1.0)
    assert np.array_equal(np.stack([pi, pj], 1), pairs)
    assert np.abs(feats - f_o).max() < 1e-5
    assert np.abs(frames - oracle_frames(dirs)).max() < 1e-13


def test_lowmodes_match_oracle(cluster):
    c, p, s, g = cluster
    rng = np.random.default_rng(3)
    f = rng.standard_normal((g.N, 3))
    rho = host(s.lowmodes(dev(f))).reshape(g.nb, 25)
    xh = g.grid["xhat"]
    w = g.grid["wnode"]
    ref = np.stack([coarse.restrict(f[g.sphere_nodes(k)], xh, w) for k in range(g.nb)])
    assert_close(rho, ref, 1e-12)
    back = host(s.lowmodes_synth(dev(ref))).reshape(g.N, 3)
    refb = np.concatenate([coarse.prolong(ref[k], xh) for k in range(g.nb)])
    assert_close(back, refb, 1e-12)


def _dataset(rng, B):
    data, ts = [], B.TrainingSet(2)
    for seed, n in ((31, 7), (32, 9)):
        c = small_cluster(n, 6.8, 0.05, seed)
        g = Geometry(c, 3, near_gap=1.0)
        pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
        xi = rng.standard_normal((2, g.nb, 25))
        t = rng.standard_normal((2, g.nb, 25))
        data.append(dict(pairs=pairs, feats=feats, dirs=dirs, xi=xi, t=t))
        ts.add(pairs[:, 0], pairs[:, 1], feats, oracle_frames(dirs), xi.transpose(1, 0, 2), t.transpose(1, 0, 2))
    return data, ts


def test_mlp_loss_and_gradient_match_oracle():
    B = _bie()
    rng = np.random.default_rng(5)
    data, ts = _dataset(rng, B)
    w = mlp.init_weights(11, out_scale=0.3)
    L, g = mlp.loss_and_grad(w, data)
    # the oracle sees the float32 inputs the kernels see
    w32 = w.astype(np.float32)
    Lg, gg = ts.eval(w32)
    assert abs(Lg - L) / L < 1e-4, (Lg, L)
    assert np.linalg.norm(gg - g) / np.linalg.norm(g) < 1e-3
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.median(np.abs(gg[big] - g[big]) / np.abs(g[big])) < 1e-3


def test_training_kernels_reduce_the_loss():
    B = _bie()
    rng = np.random.default_rng(6)
    data, ts = _dataset(rng, B)
    # a learnable target: the correction of a fixed random network
    wt = mlp.init_weights(12, out_scale=0.5)
    for d in data:
        theta, _ = mlp.forward(wt, d["feats"])
        d["t"] = mlp.predict(d["pairs"], d["dirs"], theta, d["xi"])
    ts2 = B.TrainingSet(2)
    for d in data:
        ts2.add(d["pairs"][:, 0], d["pairs"][:, 1], d["feats"], oracle_frames(d["dirs"]), d["xi"].transpose(1, 0, 2),
                d["t"].transpose(1, 0, 2))
    w0 = mlp.init_weights(13).astype(np.float32)
    l0, _ = ts2.eval(w0)
    w1, hist = ts2.train(w0, 300, cfg_per_batch=1, lr=3e-3)
    l1, _ = ts2.eval(w1)
    assert l1 < 0.2 * l0, (l0, l1, hist[:3], hist[-3:])
    # the oracle agrees on the trained loss
    assert abs(mlp.loss_and_grad(w1.astype(np.float64), data)[0] - l1) < 1e-3 * max(l1, 1e-3)


def test_precond_mlp_application_matches_oracle(cluster):
    c, p, s, g = cluster
    B = _bie()
    w = mlp.init_weights(17, out_scale=0.2)
    s.load_precond(w.astype(np.float32))
    rng = np.random.default_rng(8)
    r = rng.standard_normal((g.N, 3))
    z = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_MLP)).reshape(g.N, 3)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    theta, _ = mlp.forward(w.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    rho = np.stack([coarse.restrict(r[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    zeta = coarse.coarse_apply(pairs, dirs, theta, rho)
    ref = m0_resistance(g, r) + np.concatenate([coarse.prolong(zeta[k], xh) for k in range(g.nb)])
    assert_close(z, ref, 1e-5)
    # the M0 part alone is exact to rounding
    z0 = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_M0)).reshape(g.N, 3)
    assert_close(z0, m0_resistance(g, r), 1e-12)


def test_precond_mlp_mobility_application_matches_oracle(cluster):
    # bordered mobility form: the learned correction acts on the density part only,
    # added to M0's output; the rigid-motion rows are M0's
    c, p, s, g = cluster
    B = _bie()
    w = mlp.init_weights(19, out_scale=0.2)
    s.load_precond(w.astype(np.float32))
    rng = np.random.default_rng(9)
    r = rng.standard_normal(3 * g.N + 6 * g.nb)
    z1 = host(s.apply_precond(B.OP_MOBILITY, dev(r), precond=B.PC_MLP))
    z0 = host(s.apply_precond(B.OP_MOBILITY, dev(r), precond=B.PC_M0))
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    theta, _ = mlp.forward(w.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    rd = r[:3 * g.N].reshape(g.N, 3)
    rho = np.stack([coarse.restrict(rd[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    zeta = coarse.coarse_apply(pairs, dirs, theta, rho)
    corr = np.concatenate([coarse.prolong(zeta[k], xh) for k in range(g.nb)])
    d = (z1[:3 * g.N] - z0[:3 * g.N]).reshape(g.N, 3)
    assert_close(d, corr, 1e-5)
    assert np.array_equal(z1[3 * g.N:], z0[3 * g.N:])


def _local_dn(g, z):
    """The self term (1/2 I + D_pv) and the near series of the double layer at z."""
    ops = Operators(g)
    return ops.self_part(z, 0.0, 1.0) + 0.5 * z + ops.near_part(z, 0.0, 1.0)


def test_precond_local_application_matches_oracle(cluster):
    # BIE_PC_LOCAL: z = z0 + P zeta(R (r - A_loc z0)), z0 = M0 r, A_loc = self + near
    c, p, s, g = cluster
    B = _bie()
    w = mlp.init_weights(23, out_scale=0.2)
    s.load_precond(w.astype(np.float32))
    rng = np.random.default_rng(10)
    r = rng.standard_normal((g.N, 3))
    z = host(s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_MLP | B.PC_LOCAL)).reshape(g.N, 3)
    z0 = m0_resistance(g, r)
    wres = r - _local_dn(g, z0)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    theta, _ = mlp.forward(w.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    rho = np.stack([coarse.restrict(wres[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    zeta = coarse.coarse_apply(pairs, dirs, theta, rho)
    ref = z0 + np.concatenate([coarse.prolong(zeta[k], xh) for k in range(g.nb)])
    assert_close(z, ref, 1e-5)
    with pytest.raises(B.BieError):
        s.apply_precond(B.OP_DN_BIE, dev(r), precond=B.PC_M0 | B.PC_LOCAL)


def _local_mobility(g, xvec):
    """The bordered mobility operator without its far field: self term, identity, near
    series and the rigid-motion rows (density rows), plus the moment rows."""
    ops = Operators(g)
    mu = xvec[:3 * g.N].reshape(g.N, 3)
    far = ops.far_part(mu, 1.0, 1.0).reshape(-1)
    return ops.apply_mobility(xvec) - np.concatenate([far, np.zeros(6 * g.nb)])


def test_precond_local_mobility_application_matches_oracle(cluster):
    # BIE_PC_LOCAL on the bordered mobility form: z = z0 + [P zeta(R (r - A_loc z0)); 0]
    # with z0 = M0 r and A_loc the self term, the near series and the bordered rows
    c, p, s, g = cluster
    B = _bie()
    w = mlp.init_weights(29, out_scale=0.2)
    s.load_precond(w.astype(np.float32))
    rng = np.random.default_rng(12)
    r = rng.standard_normal(3 * g.N + 6 * g.nb)
    z = host(s.apply_precond(B.OP_MOBILITY, dev(r), precond=B.PC_MLP | B.PC_LOCAL))
    z0 = host(s.apply_precond(B.OP_MOBILITY, dev(r), precond=B.PC_M0))
    wres = (r - _local_mobility(g, z0))[:3 * g.N].reshape(g.N, 3)
    pairs, feats, dirs = coarse.pair_features(c, g.near, 1.0)
    theta, _ = mlp.forward(w.astype(np.float32).astype(np.float64), feats.astype(np.float32).astype(np.float64))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    rho = np.stack([coarse.restrict(wres[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    zeta = coarse.coarse_apply(pairs, dirs, theta, rho)
    corr = np.concatenate([coarse.prolong(zeta[k], xh) for k in range(g.nb)])
    assert_close((z[:3 * g.N] - z0[:3 * g.N]).reshape(g.N, 3), corr, 1e-5)
    assert np.array_equal(z[3 * g.N:], z0[3 * g.N:])


def test_training_sample_mobility_local_matches_oracle(cluster):
    # bie_precond_sample on the bordered form: target = R (x - M0 b), xi = R (b - A_loc M0 b),
    # both on the density part
    c, p, s, g = cluster
    B = _bie()
    rng = np.random.default_rng(13)
    b = rng.standard_normal(3 * g.N + 6 * g.nb)
    x = rng.standard_normal(3 * g.N + 6 * g.nb)
    xi, t = s.precond_sample(B.OP_MOBILITY, B.PC_M0 | B.PC_LOCAL, dev(b), dev(x))
    z0 = host(s.apply_precond(B.OP_MOBILITY, dev(b), precond=B.PC_M0))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    dens = lambda v: v[:3 * g.N].reshape(g.N, 3)
    R = lambda f: np.stack([coarse.restrict(f[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    assert_close(host(t).reshape(g.nb, 25), R(dens(x - z0)), 1e-11)
    assert_close(host(xi).reshape(g.nb, 25), R(dens(b - _local_mobility(g, z0))), 1e-11)


@pytest.mark.parametrize("local", [False, True])
def test_training_sample_matches_oracle(cluster, local):
    # bie_precond_sample: target = R x - R M0 b, xi = R b or R (b - A_loc M0 b)
    c, p, s, g = cluster
    B = _bie()
    rng = np.random.default_rng(11)
    b = rng.standard_normal((g.N, 3))
    x = rng.standard_normal((g.N, 3))
    xi, t = s.precond_sample(B.OP_DN_BIE, B.PC_M0 | (B.PC_LOCAL if local else 0), dev(b), dev(x))
    xh, wq = g.grid["xhat"], g.grid["wnode"]
    z0 = m0_resistance(g, b)
    R = lambda f: np.stack([coarse.restrict(f[g.sphere_nodes(k)], xh, wq) for k in range(g.nb)])
    assert_close(host(t).reshape(g.nb, 25), R(x) - R(z0), 1e-11)
    ref_xi = R(b - _local_dn(g, z0)) if local else R(b)
    assert_close(host(xi).reshape(g.nb, 25), ref_xi, 1e-11)


def test_nonfinite_weights_are_rejected(cluster):
    c, p, s, g = cluster
    B = _bie()
    w = np.zeros(B.mlp_n_weights(), np.float32)
    w[5] = np.nan
    with pytest.raises(B.BieError):
        s.load_precond(w)


def test_trained_network_gain_over_m0():
    # committed weights (paper_1707_06551_amd/weights/precond_dn.npz, trained on the GPU
    # from plain float64 solves of 64-sphere, p = 16 configurations); held-out seeds
    # that neither training, validation nor the relaxation choice used
    from paper_1707_06551_amd.inputs import make_workload
    from paper_1707_06551_amd.precond_train import load_weights
    B = _bie()
    w, meta = load_weights()
    m0, ml, mix = [], [], []
    for sd in (700000, 700001):
        wk = make_workload("spheres64_p16_train", seed=sd)
        s = B.Spheres(wk["centres"], 16, near_gap=1.0)
        s.load_precond(w)
        F0, T0, _, i0 = s.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precond=B.PC_M0)
        F1, T1, _, i1 = s.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precond=B.PC_MLP)
        F2, T2, _, i2 = s.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precision=B.MIXED, precond=B.PC_MLP)
        assert i0["converged"] and i1["converged"] and i2["converged"]
        assert i1["fallback_used"] == 0
        assert_close(F1, F0, 1e-6)
        assert_close(F2, F0, 1e-6)
        m0.append(i0["iters"])
        ml.append(i1["iters"])
        mix.append(i2["iters"])
        s.close()
    print(f"GMRES iterations M0 {m0}, learned {ml}, mixed+learned {mix}")
    assert sum(ml) <= 0.9 * sum(m0), (m0, ml)


def test_trained_network_gain_over_m0_mobility():
    # committed weights for the bordered mobility form (weights/precond_mob.npz, trained
    # from plain float64 solves of 64-sphere, p = 12 configurations at volume fraction
    # 0.25 with low-mode slip); held-out seeds of the active-slip mobility problem
    import os
    from paper_1707_06551_amd.inputs import make_workload, slip_field
    from paper_1707_06551_amd.precond_train import DEFAULT_FILES, load_weights
    B = _bie()
    if not os.path.exists(DEFAULT_FILES["mob"]):
        pytest.skip("no trained mobility weights")
    w, meta = load_weights(DEFAULT_FILES["mob"])
    m0, ml, mix = [], [], []
    for sd in (700000, 700001):
        wk = make_workload("spheres64_p12_slip_train", seed=sd)
        s = B.Spheres(wk["centres"], 12, near_gap=1.0)
        s.load_precond(w)
        xyz, _ = s.nodes()
        sphere_of = np.arange(s.N) // s.P
        slip = dev(slip_field(wk["slip_coef"], xyz - wk["centres"][sphere_of], sphere_of))
        v0, o0, _, i0 = s.solve_mobility(wk["F"], wk["T"], slip=slip, tol=1e-8, precond=B.PC_M0)
        v1, o1, _, i1 = s.solve_mobility(wk["F"], wk["T"], slip=slip, tol=1e-8, precond=B.PC_MLP)
        v2, o2, _, i2 = s.solve_mobility(wk["F"], wk["T"], slip=slip, tol=1e-8, precision=B.MIXED,
                                         precond=B.PC_MLP)
        assert i0["converged"] and i1["converged"] and i2["converged"]
        assert i1["fallback_used"] == 0
        for v, o in ((v1, o1), (v2, o2)):
            assert_close(v, v0, 1e-6)
            assert_close(o, o0, 1e-6)
        m0.append(i0["iters"])
        ml.append(i1["iters"])
        mix.append(i2["iters"])
        s.close()
    print(f"mobility GMRES iterations M0 {m0}, learned {ml}, mixed+learned {mix}")
    # M0 already converges in about 40 iterations on this form and the low-mode part of
    # the error is not what limits it: the trained correction gains a few percent (the
    # relaxation scan stored with the weights); it must never cost iterations
    assert sum(ml) <= sum(m0), (m0, ml)


def test_bad_network_falls_back_to_plain_gmres():
    # a network scaled far beyond its relaxation stalls the preconditioned solve; the
    # solver must notice, restart plain float64 GMRES from the current iterate, converge
    from paper_1707_06551_amd.inputs import make_workload
    from paper_1707_06551_amd.precond_train import load_weights, scaled
    B = _bie()
    w, meta = load_weights()
    wk = make_workload("spheres64_p16_train", seed=700002)
    s = B.Spheres(wk["centres"], 8, near_gap=1.0)
    s.load_precond(scaled(w, 200.0))
    F, T, _, info = s.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precond=B.PC_MLP, max_iter=2000)
    F0, T0, _, i0 = s.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precond=B.PC_NONE)
    assert info["converged"] and info["fallback_used"] == 1, info
    assert_close(F, F0, 1e-6)
    s.close()
