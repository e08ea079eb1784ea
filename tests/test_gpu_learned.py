"""Learned troubled-cell indicator on the GPU (through the C ABI) against the
FP64 reference in oracle/mlp.py and the FP64 scheme oracle.

Tolerances: MFMA GEMM within the FP32 summation bound; features within one
BF16 rounding (2^-8 relative) plus 1e-6; network outputs and gradients at
BF16 level (2-3 %), since the kernels round activations and gradients to
BF16; decisions identical to the GPU forward pass except within 1e-5 of a
band edge, and to the FP64 reference except within 0.03; the scheme with
the learned flags within 1e-12 of the oracle given the same flags."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2201_12193_amd import inputs as I
from tests.parity_util import comp_scale, rel_state_err, kxrcf_flags, MISMATCHES_ALLOWED

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bf16(P):
    import torch
    return _t(np.asarray(P, dtype=np.float32)).to(torch.bfloat16)


def _params(seed=0, b3=0.0):
    from paper_2201_12193_amd.indicator import init_params, OFF_B3
    P = init_params(seed).astype(np.float64)
    P[OFF_B3] = b3
    return mlp.bf16_round(P)


def _state(seed=7, n=64, bc=I.PERIODIC, steps=2):
    prob, U, _ = I.euler_quadrants_2d(seed=seed, n=n, nq=2)
    prob = prob.replace(bc_x=bc, bc_y=bc)
    for _ in range(steps):
        U = oracle.rk3_step(prob, U, oracle.dt(prob, U))
    return prob, U


def _gpu_z(solver, U, P, n):
    """Logits of every interior cell through the training forward pass."""
    import torch
    from paper_2201_12193_amd.mrhweno import mlp_cache_bytes, mlp_forward
    cells = torch.arange(n, dtype=torch.int32, device="cuda")
    X = solver.features(0, _t(U), cells)
    pad = (-n) % 16
    if pad:
        X = torch.cat([X, torch.zeros((pad, X.shape[1]), dtype=X.dtype, device=X.device)])
    cache = torch.empty(mlp_cache_bytes(X.shape[0]) + 256, dtype=torch.uint8, device="cuda")
    z = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
    mlp_forward(X, _bf16(P), cache, z)
    torch.cuda.synchronize()
    return X[:n], z[:n].cpu().numpy().astype(np.float64)


def _learned_solver(prob, U, P, lo=0.2, hi=0.8):
    from paper_2201_12193_amd.mrhweno import Solver
    prob = prob.replace(tc_mode=I.TC_LEARNED)
    Ut = _t(U)
    s = Solver([prob], [Ut])
    s.set_indicator(_bf16(P), lo, hi)
    return s, Ut, prob


def _centred_params(prob, U, seed=0):
    """Random network with W3 scaled and b3 chosen so that the logits of
    the state's cells spread over about [-3, 3] around 0."""
    from paper_2201_12193_amd.mrhweno import Solver
    from paper_2201_12193_amd.indicator import OFF_B3, OFF_W3
    P = _params(seed)
    s = Solver([prob], [_t(U)])
    _, z = _gpu_z(s, U, P, prob.ncell)
    s.close()
    q20, q80 = np.percentile(z, [20, 80])
    k = 3.0 / max(float(q80 - q20), 1e-6)
    P[OFF_W3:OFF_B3] = mlp.bf16_round(k * P[OFF_W3:OFF_B3])
    P[OFF_B3] = float(mlp.bf16_round([-k * (np.median(z) - P[OFF_B3])])[0])
    return P


# ------------------------------------------------------------------ kernels
@pytest.mark.parametrize("M,N,K,trans", [(16, 16, 32, False), (37, 53, 75, False), (64, 320, 300, True),
                                         (200, 64, 4096, True)])
def test_mfma_gemm_matches_fp64(M, N, K, trans):
    """The GEMM kernel's MFMA lane layout and strides: C = A B."""
    import torch
    from paper_2201_12193_amd.mrhweno import mlp_gemm
    g = torch.Generator().manual_seed(M * 1000 + N)
    A = torch.randn((K, M) if trans else (M, K), generator=g).to(torch.bfloat16)
    B = torch.randn((K, N), generator=g).to(torch.bfloat16)
    Ad = A.cuda().t() if trans else A.cuda()
    C = mlp_gemm(Ad, B.cuda()).cpu().double().numpy()
    A64 = (A.t() if trans else A).double().numpy()
    B64 = B.double().numpy()
    ref = A64 @ B64
    bound = K * 2.0 ** -23 * (np.abs(A64) @ np.abs(B64))
    assert np.all(np.abs(C - ref) <= bound + 1e-30)


@pytest.mark.parametrize("bc", [I.PERIODIC, I.TRANSMISSIVE, I.REFLECTIVE])
def test_features_match_oracle(bc):
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    prob, U = _state(seed=21, n=40, bc=bc, steps=1)
    rng = np.random.default_rng(4)
    cells = np.unique(np.concatenate([[0, 39, 40 * 39, 40 * 40 - 1, 41, 20 * 40 + 19],
                                      rng.choice(prob.ncell, 200, replace=False)])).astype(np.int32)
    s = Solver([prob], [_t(U)])
    X = s.features(0, _t(U), torch.from_numpy(cells).cuda()).float().cpu().numpy().astype(np.float64)
    s.close()
    ref = mlp.features(prob, U, cells)
    err = np.abs(X - ref) - (2.0 ** -8 * np.abs(ref) + 1e-6)
    assert err.max() <= 0.0, float(err.max())


def test_forward_backward_match_oracle():
    """Logits, loss and every gradient block of the MFMA training kernels
    against the FP64 reference on the same BF16 features and weights."""
    import torch
    from paper_2201_12193_amd.mrhweno import Solver, mlp_backward, mlp_cache_bytes, mlp_forward, MLP_PARAMS
    prob, U = _state(seed=23, n=48, steps=2)
    s = Solver([prob], [_t(U)])
    rng = np.random.default_rng(8)
    B = 512
    cells = rng.choice(prob.ncell, B, replace=False).astype(np.int32)
    X = s.features(0, _t(U), torch.from_numpy(cells).cuda())
    s.close()
    y = (rng.random(B) < 0.5).astype(np.float32)
    P = _params(3, b3=0.1)
    Pd = _bf16(P)
    cache = torch.empty(mlp_cache_bytes(B) + 256, dtype=torch.uint8, device="cuda")
    z = torch.empty(B, dtype=torch.float32, device="cuda")
    grads = torch.empty(MLP_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(B, dtype=torch.float32, device="cuda")
    yd = _t(y)
    mlp_forward(X, Pd, cache, z)
    mlp_backward(X, Pd, cache, yd, grads, loss)
    torch.cuda.synchronize()
    X64 = X.float().cpu().numpy().astype(np.float64)
    # the network hands the first hidden layer to the second in BF16
    zr, _ = mlp.forward(X64, P, bf16_hidden=True)
    zg = z.cpu().numpy()
    zs = np.abs(zr).mean() + 1e-3
    # FP32 sums differ from FP64 in the last bits, which now and then moves a
    # hidden value across a BF16 rounding boundary (one BF16 unit of one term)
    w = mlp.unpack(P)
    _, a64 = mlp.forward(X64, P, bf16_hidden=True)
    ulp_bound = 2.0 ** -7 * (a64["h1"] @ (np.abs(w["W2"]).T @ np.abs(w["W3"])))
    dz = np.abs(zg - zr)
    assert np.all(dz <= 1e-4 * zs + ulp_bound), float((dz - ulp_bound).max())
    assert (dz > 1e-4 * zs).sum() <= 0.02 * B
    assert float(loss.mean()) == pytest.approx(float(np.mean(mlp.bce(zr, y))), rel=1e-3)
    # the plain FP64 network is within BF16 level of it
    z64, _ = mlp.forward(X64, P)
    assert np.abs(z64 - zr).max() <= 0.03 * zs
    gr = mlp.gradient(X64, P, y, bf16_hidden=True)
    # FP32 logits move the back-propagated dz by up to dzmax / 4
    dzmax = float(np.abs(zg - zr).max())
    gabs = _abs_gradient(X64, P, y)
    gdz = _abs_gradient(X64, P, y, dz=np.full(B, 0.25 * dzmax / B))
    gg = grads.cpu().numpy().astype(np.float64)
    for name, (a, b) in {"W1": (mlp.OFF["W1"], mlp.OFF["b1"]), "b1": (mlp.OFF["b1"], mlp.OFF["W2"]),
                         "W2": (mlp.OFF["W2"], mlp.OFF["b2"]), "b2": (mlp.OFF["b2"], mlp.OFF["W3"]),
                         "W3": (mlp.OFF["W3"], mlp.OFF["b3"]), "b3": (mlp.OFF["b3"], mlp.OFF["b3"] + 1)}.items():
        # BF16 rounding of activations and back-propagated gradients, measured
        # against the sum of the magnitudes of the terms of each gradient
        err = np.abs(gg[a:b] - gr[a:b]) - (2.0 ** -6 * gabs[a:b] + 2.0 * gdz[a:b] + 1e-12)
        assert err.max() <= 0.0, (name, float(err.max()))
        assert np.linalg.norm(gg[a:b] - gr[a:b]) <= 0.1 * np.linalg.norm(gr[a:b]), name
    assert np.all(gg[mlp.OFF["b3"] + 1:] == 0.0)


def _abs_gradient(X, P, y, dz=None):
    """The gradient's chain rule with every term replaced by its magnitude
    (the scale of the rounding error of each gradient entry); dz, if given,
    replaces |d loss / d z|."""
    w = {k: np.abs(v) for k, v in mlp.unpack(P).items()}
    z, a = mlp.forward(X, P)
    if dz is None:
        dz = np.abs(mlp.sigmoid(z) - y) / X.shape[0]
    # a pre-activation within rounding of zero may pass the ReLU on one side
    on2 = a["a2"] > -0.02 * np.abs(a["a2"]).mean()
    on1 = a["a1"] > -0.02 * np.abs(a["a1"]).mean()
    g = np.zeros(mlp.NPARAM)
    g[mlp.OFF["W3"]:mlp.OFF["b3"]] = np.abs(a["a2"] * on2).T @ dz
    g[mlp.OFF["b3"]] = dz.sum()
    d2 = np.outer(dz, w["W3"]) * on2
    g[mlp.OFF["W2"]:mlp.OFF["b2"]] = (d2.T @ np.abs(a["a1"] * on1)).ravel()
    g[mlp.OFF["b2"]:mlp.OFF["W3"]] = d2.sum(axis=0)
    d1 = (d2 @ w["W2"]) * on1
    g[mlp.OFF["W1"]:mlp.OFF["b1"]] = (d1.T @ np.abs(X)).ravel()
    g[mlp.OFF["b1"]:mlp.OFF["W2"]] = d1.sum(axis=0)
    return g


def test_adam_matches_oracle():
    import torch
    from paper_2201_12193_amd.mrhweno import mlp_adam, MLP_PARAMS
    rng = np.random.default_rng(12)
    w = rng.standard_normal(MLP_PARAMS).astype(np.float32)
    m = (0.01 * rng.standard_normal(MLP_PARAMS)).astype(np.float32)
    v = (1e-4 * rng.random(MLP_PARAMS)).astype(np.float32)
    g = (0.1 * rng.standard_normal(MLP_PARAMS)).astype(np.float32)
    wd, md, vd, gd = _t(w), _t(m), _t(v), _t(g)
    pd = torch.empty(MLP_PARAMS, dtype=torch.bfloat16, device="cuda")
    mlp_adam(wd, pd, gd, md, vd, 3, 1e-3)
    torch.cuda.synchronize()
    # the kernel takes the hyper-parameters in FP32
    f32 = lambda x: float(np.float32(x))
    wr, mr, vr = mlp.adam(w.astype(np.float64), g.astype(np.float64), m.astype(np.float64),
                          v.astype(np.float64), 3, f32(1e-3), f32(0.9), f32(0.999), f32(1e-8))
    assert np.allclose(wd.cpu().numpy(), wr, rtol=1e-6, atol=1e-7)
    # FP32 rounding of the two terms of each moment update
    # FP32 rounding of the two terms of each moment update
    assert np.all(np.abs(md.cpu().numpy() - mr) <= 1e-6 * (0.9 * np.abs(m) + 0.1 * np.abs(g)))
    assert np.all(np.abs(vd.cpu().numpy() - vr) <= 1e-6 * (0.999 * v + 0.001 * g.astype(np.float64) ** 2))
    assert np.array_equal(pd.float().cpu().numpy().astype(np.float64), mlp.bf16_round(wd.cpu().numpy()))


# ------------------------------------------------------------- fused path
@pytest.mark.parametrize("bc,beta_on", [(I.PERIODIC, 0), (I.REFLECTIVE, 0), (I.PERIODIC, 1)])
def test_indicator_decisions_and_flags(bc, beta_on):
    """Fused inference decisions against the training forward pass (same
    BF16 arithmetic) and the FP64 reference; band cells get the KXRCF flag
    (with beta on q or on p, the fallback's two variants).  Reflective
    walls exercise the fused kernel's mirrored ghost staging."""
    import torch
    prob, U = _state(seed=31, n=64, bc=bc, steps=2)
    prob = prob.replace(beta_on=beta_on)
    P = _centred_params(prob, U)
    lo, hi = 0.3, 0.7
    s, Ut, pl = _learned_solver(prob, U, P, lo, hi)
    dec, fl = s.indicator(0, _t(U))
    dec = dec.cpu().numpy().ravel()
    fl = fl.cpu().numpy().ravel()
    _, z = _gpu_z(s, U, P, prob.ncell)
    s.close()
    sg = 1.0 / (1.0 + np.exp(-z))
    want = np.where(sg > hi, 1, np.where(sg < lo, 0, 2))
    near = (np.abs(sg - lo) < 1e-5) | (np.abs(sg - hi) < 1e-5)
    assert np.all((dec == want) | near)
    assert (dec == 0).sum() > 100 and (dec == 1).sum() > 100 and (dec == 2).sum() > 20
    # FP64 reference
    Xr = mlp.features(prob, U, np.arange(prob.ncell))
    sr = mlp.sigmoid(mlp.forward(Xr, P)[0])
    wr = np.where(sr > hi, 1, np.where(sr < lo, 0, 2))
    near_r = (np.abs(sr - lo) < 0.03) | (np.abs(sr - hi) < 0.03)
    assert np.all((dec == wr) | near_r)
    # final flags: the decision where confident, KXRCF in the band
    _, fk, num, den = oracle.reconstruct(prob.replace(tc_mode=I.TC_KXRCF), U)
    fk, num, den = fk.ravel(), num.ravel(), den.ravel()
    conf = dec != 2
    assert np.array_equal(fl[conf], dec[conf])
    tag = "learned/band_fallback"
    n, out = kxrcf_flags(tag, prob, fl[~conf], fk[~conf], num[~conf], den[~conf], comp_scale(prob, U)[0])
    assert out == 0 and n <= MISMATCHES_ALLOWED.get(tag, 0), (n, out)


def _wrap(f):
    return np.pad(np.asarray(f).astype(np.uint8), 2, mode="wrap")


def test_learned_residual_matches_oracle():
    prob, U = _state(seed=33, n=64, steps=2)
    P = _centred_params(prob, U, seed=1)
    s, Ut, pl = _learned_solver(prob, U, P)
    R, fl = s.residual(0, _t(U))
    _, fl2 = s.indicator(0, _t(U))
    s.close()
    fl = fl.cpu().numpy()
    assert np.array_equal(fl, fl2.cpu().numpy())
    assert fl.sum() > 0
    ref = oracle.residual_given(prob, U, _wrap(fl))
    sc = comp_scale(prob, U)
    dR = np.abs(R.cpu().numpy() - ref).reshape(prob.ncomp, -1).max(axis=1) / (sc / oracle.dt(prob, U))
    assert dR.max() <= TOL, dR


def _oracle_step_given(prob, U, dt, flag_fn):
    """SSP-RK3 step of the oracle with the troubled-cell map of each stage
    input taken from flag_fn (modified stage inputs kept, U^n included)."""
    def stage(V):
        f = flag_fn(V)
        return oracle.residual_given(prob, V, _wrap(f)), oracle.modify(prob, V, f.ravel())
    L, Un = stage(U)
    U1 = Un + dt * L
    L, U1t = stage(U1)
    U2 = 3.0 / 4.0 * Un + 1.0 / 4.0 * U1t + 1.0 / 4.0 * dt * L
    L, U2t = stage(U2)
    return 1.0 / 3.0 * Un + 2.0 / 3.0 * U2t + 2.0 / 3.0 * dt * L


def test_learned_steps_match_oracle():
    prob, U = _state(seed=35, n=48, steps=1)
    P = _centred_params(prob, U, seed=2)
    s, Ut, pl = _learned_solver(prob, U, P)
    # a second context on the same weights evaluates the flags of oracle stage inputs
    s2, _, _ = _learned_solver(prob, U, P)

    def flag_fn(V):
        return s2.indicator(0, _t(V))[1].cpu().numpy()

    sc = comp_scale(prob, U)
    prev = U.copy()
    for k in range(3):
        s.step(1)
        dt = s.last_dt()[0]
        s.sync()
        got = Ut.cpu().numpy()
        assert dt == oracle.dt(prob, prev)
        ref = _oracle_step_given(prob, prev, dt, flag_fn)
        e = rel_state_err(prob, got, ref, sc)
        assert e <= TOL, (k, e)
        prev = got
    s.close()
    s2.close()


def test_learned_batched_graph_equals_eager():
    """A batch mixing learned and KXRCF instances: graph replay and eager
    launches agree bit for bit, and the KXRCF instance equals its
    standalone run."""
    import torch
    from paper_2201_12193_amd.mrhweno import Solver
    pa, Ua = _state(seed=41, n=64, steps=0)
    pb, Ub = _state(seed=42, n=48, steps=0)
    pc, Uc = _state(seed=43, n=40, bc=I.TRANSMISSIVE, steps=0)
    P = _centred_params(pa, Ua, seed=4)
    pa, pc = pa.replace(tc_mode=I.TC_LEARNED), pc.replace(tc_mode=I.TC_LEARNED)
    probs = [pa, pb, pc]
    states = []
    for mode in ("graph", "eager"):
        Us = [_t(Ua), _t(Ub), _t(Uc)]
        s = Solver(probs, Us)
        s.set_indicator(_bf16(P))
        if mode == "graph":
            s.step(4)
        else:
            s.profile(4)
        s.sync()
        states.append([u.cpu().numpy() for u in Us])
        s.close()
    for a, b in zip(*states):
        assert np.array_equal(a, b)
    Ut = _t(Ub)
    s = Solver([pb], [Ut])
    s.step(4)
    s.sync()
    assert np.array_equal(Ut.cpu().numpy(), states[0][1])
    s.close()


def test_learned_batch_mixing_beta_variants():
    """Learned instances with beta on q and on p in one batch: the fallback
    launches one kernel per variant, each skipping the other's band cells;
    every instance ends bit for bit where it ends alone."""
    from paper_2201_12193_amd.mrhweno import Solver
    pa, Ua = _state(seed=45, n=64, steps=1)
    pb, Ub = _state(seed=46, n=56, steps=1)
    P = _centred_params(pa, Ua, seed=5)
    pa = pa.replace(tc_mode=I.TC_LEARNED)
    pb = pb.replace(tc_mode=I.TC_LEARNED, beta_on=1)
    Us = [_t(Ua), _t(Ub)]
    s = Solver([pa, pb], Us)
    s.set_indicator(_bf16(P))
    s.step(3)
    s.sync()
    both = [u.cpu().numpy() for u in Us]
    s.close()
    for prob, U0, got in ((pa, Ua, both[0]), (pb, Ub, both[1])):
        Ut = _t(U0)
        s = Solver([prob], [Ut])
        s.set_indicator(_bf16(P))
        s.step(3)
        s.sync()
        assert np.array_equal(Ut.cpu().numpy(), got)
        s.close()


def test_learned_requires_weights():
    from paper_2201_12193_amd.mrhweno import Solver, MrError, ERR_NOT_READY
    prob, U = _state(seed=45, n=32, steps=0)
    s = Solver([prob.replace(tc_mode=I.TC_LEARNED)], [_t(U)])
    with pytest.raises(MrError) as e:
        s.step(1)
    assert e.value.status == ERR_NOT_READY
    with pytest.raises(MrError) as e:
        s.indicator(0, _t(U))
    assert e.value.status == ERR_NOT_READY
    s.close()


# ------------------------------------------------------------ training
def test_training_reduces_loss():
    """A short GPU training run on KXRCF labels of the solver's own run."""
    from paper_2201_12193_amd.indicator import collect, train, evaluate
    X, y, stats = collect([(5, 128, 40, 20)], seed=0, log=lambda *a, **k: None)
    assert stats["positives"] > 50
    P, hist = train(X, y, steps=400, batch=1024, lr=2e-3, log=lambda *a, **k: None, log_every=50)
    assert hist[0][0] == 1 and hist[-1][1] < 0.5 * hist[0][1], hist
    ev = evaluate(P, X, y)
    assert ev["accuracy_confident"] > 0.9, ev
