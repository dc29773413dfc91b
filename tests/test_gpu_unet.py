"""GPU parity of the warm-start network kernels against the FP64 oracle
reference given the same BF16-rounded operands (FP32 accumulation only:
relative error 1e-5), and of the whole network's forward pass and gradients
(BF16 activations between layers: looser bounds)."""
import ctypes
import math

import numpy as np
import pytest

from oracle import unet as U

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def bf16_bits(x):
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return u.astype(np.uint16)


def bf16_round(x):
    return (bf16_bits(x).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def dev_bits(bits):
    return torch.from_numpy(bits.view(np.int16).copy()).cuda()


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def P():
    import paper_2604_15434_amd as P

    return P


def _conv(P, mode, n, cin, cout, x=None, dy=None, w=None, b=None):
    L = P._lib
    out_n = {0: n**3 * cout, 1: n**3 * cin, 2: 27 * cin * cout, 4: n**3}[mode]
    out = torch.zeros(out_n, dtype=torch.float32, device="cuda")
    wb = (54 * ((cin + 15) // 16 * 16) * ((cout + 15) // 16 * 16) + 255) // 256 * 256
    wsz = 2 * wb + 4 * 240 * (27 * cin * cout + cout)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    wd = torch.from_numpy(w.astype(np.float32)).cuda()
    bd = torch.from_numpy(b.astype(np.float32)).cuda() if b is not None else None
    xd = dev_bits(bf16_bits(x)) if x is not None else None
    yd = dev_bits(bf16_bits(dy)) if dy is not None else None
    ptr = lambda t: ctypes.c_void_p(t.data_ptr() if t is not None else 0)  # noqa: E731
    rc = L.lib().ws_conv3(mode, n, cin, cout, ptr(xd), ptr(yd), ptr(wd), ptr(bd), ptr(out), ptr(ws), wsz,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n,cin,cout", [(16, 16, 16), (16, 48, 16), (32, 96, 32), (16, 32, 64), (16, 16, 48), (16, 32, 96), (64, 16, 16), (64, 48, 16), (64, 32, 64), (64, 16, 32), (64, 64, 64), (64, 96, 32), (128, 16, 16)])
def test_conv_forward_matches_reference(P, n, cin, cout):
    """Every forward kernel form: the one-plane and LDS-staged ones (n not a
    multiple of 64, or more than 48 input channels), and the plane march
    with 16, 32 and 48 input channels, one and several output tiles, and
    8- and 32-plane tiles (64^3, 128^3)."""
    rng = np.random.default_rng(cin + cout)
    x = rng.standard_normal((n, n, n, cin))
    w = rng.standard_normal((27, cin, cout)) * 0.1
    b = rng.standard_normal(cout)
    got = _conv(P, 0, n, cin, cout, x=x, w=w, b=b).reshape(n, n, n, cout)
    ref = U.conv3(bf16_round(x), bf16_round(w), b.astype(np.float32).astype(np.float64))
    assert rel(got, ref) < 1e-5


@pytest.mark.parametrize("n,cin,cout", [(16, 16, 16), (16, 48, 16), (16, 32, 64), (16, 4, 16), (32, 96, 32), (64, 16, 16), (64, 32, 16), (64, 16, 32), (64, 16, 64)])
def test_conv_input_and_weight_gradients(P, n, cin, cout):
    rng = np.random.default_rng(7 * cin + cout)
    x = rng.standard_normal((n, n, n, cin))
    dy = rng.standard_normal((n, n, n, cout))
    w = rng.standard_normal((27, cin, cout)) * 0.1
    xb, dyb, wb = bf16_round(x), bf16_round(dy), bf16_round(w)
    dx_ref, dw_ref, _ = U.conv3_backward(xb, wb, dyb)
    if cin % 16 == 0:
        dx = _conv(P, 1, n, cin, cout, dy=dy, w=w).reshape(n, n, n, cin)
        assert rel(dx, dx_ref) < 1e-5
    dw = _conv(P, 2, n, cin, cout, x=x, dy=dy, w=w).reshape(27, cin, cout)
    assert rel(dw, dw_ref) < 1e-5
    # fixed-order reduction: a second run is bitwise identical
    dw2 = _conv(P, 2, n, cin, cout, x=x, dy=dy, w=w).reshape(27, cin, cout)
    assert np.array_equal(dw, dw2)


def _ref_params(flat):
    p, o = {}, 0
    for (name, ci, co) in U.LAYERS:
        p[name + ".w"] = flat[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        p[name + ".b"] = flat[o:o + co]
        o += co
    p["head.w"] = flat[o:o + 16]
    p["head.b"] = flat[o + 16:o + 17]
    return p


def _net_case(n=64, seed=5):
    from workloads import lognormal_density

    rho = lognormal_density(n, 125.0 * n / 64, seed=seed)
    prm = dict(omega_m0=0.3071, alpha_b0=-0.5, alpha_m0=0.1, a=0.8)
    return rho, prm


def test_network_forward_and_loss_track_reference(P):
    """Whole network on a 64^3 lognormal density: BF16 activations between
    layers, so the prediction and the training loss are compared with the
    FP64 network at 3e-2 relative."""
    import oracle
    from paper_2604_15434_amd.warmstart import WarmStart

    n = 64
    rho, prm = _net_case(n)
    net = WarmStart(seed=3)
    p = _ref_params(net.params.cpu().numpy().astype(np.float64))
    x0 = U.input_features(rho, prm["alpha_b0"], prm["alpha_m0"], prm["a"])
    y_ref, _ = U.forward(p, x0, keep=False)
    rho_d = torch.from_numpy(rho).cuda()
    yhat = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    net.predict(rho_d, prm, yhat)
    got = yhat.cpu().numpy().reshape(n, n, n).astype(np.float64)
    assert rel(got, y_ref) < 3e-2
    y_tr = torch.zeros_like(yhat)
    net.forward_train(rho_d, prm, y_tr)
    assert rel(y_tr.cpu().numpy().reshape(n, n, n).astype(np.float64), y_ref) < 3e-2
    c = oracle.eft_coefficients(**prm)
    chi = _smooth_chi(n)
    t_ref = U.source_target(chi, rho, c["s"] * c["mu_chi"])
    loss = net.train_step(rho_d, torch.from_numpy(chi).cuda(), prm, 0.0)
    assert loss == pytest.approx(np.mean((y_ref - t_ref) ** 2), rel=3e-2)


def _smooth_chi(n):
    rng = np.random.default_rng(11)
    k2 = np.add.outer(np.add.outer(np.fft.fftfreq(n)**2, np.fft.fftfreq(n)**2), np.fft.fftfreq(n)**2)
    return np.real(np.fft.ifftn(np.fft.fftn(rng.standard_normal((n, n, n))) * np.exp(-k2 * 200.0))) * 1e-3


# tensors of the training workspace: index -> (name, channels, grid level)
_T = ["x0", "a1", "c1", "p1", "a2", "c2", "p2", "a3", "b3", "a4", "b4", "a5", "b5"]
_T_CH = [16, 16, 48, 16, 32, 96, 32, 64, 64, 32, 32, 16, 16]
_T_LEVEL = [0, 0, 0, 1, 1, 1, 2, 2, 2, 1, 1, 0, 0]


def _read(net, n, t, gradient=False):
    m = n >> _T_LEVEL[t]
    out = torch.empty(m**3 * _T_CH[t], dtype=torch.float32, device="cuda")
    net.tensor(n, t, out, gradient=gradient)
    return out.cpu().numpy().astype(np.float64).reshape(m, m, m, _T_CH[t])


def test_network_backward_stages_match_reference(P):
    """ws_unet_backward on a 64^3 lognormal density, checked stage by stage:
    each layer's parameter gradients and output gradient are recomputed by the
    FP64 reference from that layer's own input -- the BF16 activations and
    the BF16 gradient the network stored (read back from the training
    workspace) -- with the same BF16 weights, and the reference rounds the
    gradient it hands on to BF16 as the kernels store it.  Weight and bias
    gradients within 1e-5 relative (FP32 accumulation only), handed-on
    activation gradients within 1e-4 relative L2 (BF16 roundings that FP32
    accumulation flips).  Chaining the stages instead lets those flips grow
    to a BF16 ulp (4e-3) over the ten layers, so the stages are compared
    separately."""
    from paper_2604_15434_amd.warmstart import WarmStart

    n = 64
    rho, prm = _net_case(n)
    net = WarmStart(seed=3)
    p = _ref_params(net.params.cpu().numpy().astype(np.float64))
    pb = {k: (bf16_round(v) if k.endswith(".w") and not k.startswith("head") else v) for k, v in p.items()}
    rho_d = torch.from_numpy(rho).cuda()
    net.forward_train(rho_d, prm)
    act = {name: _read(net, n, t) for t, name in enumerate(_T)}
    act["x0"] = act["x0"][..., :4]
    rng = np.random.default_rng(21)
    dy = (rng.standard_normal(n**3) * 2.0 / n**3).astype(np.float32)
    grads = torch.zeros(net.params.numel(), dtype=torch.float32, device="cuda")
    net.backward(torch.from_numpy(dy).cuda(), n, grads)
    grad = {name: _read(net, n, t, gradient=True) for t, name in enumerate(_T) if t > 0}
    g = grads.cpu().numpy().astype(np.float64)
    gsl, o = {}, 0
    for (name, ci, co) in U.LAYERS:
        gsl[name + ".w"] = g[o:o + 27 * ci * co].reshape(27, ci, co)
        o += 27 * ci * co
        gsl[name + ".b"] = g[o:o + co]
        o += co
    gsl["head.w"], gsl["head.b"] = g[o:o + 16], g[o + 16:o + 17]
    errs = {}

    def cmp(key, got, ref):
        errs[key] = rel(got, ref)

    # head: d b5 = bf16(dy hw), masked by the ReLU of l5b
    dyn = dy.astype(np.float64).reshape(n, n, n)
    cmp("head.w", gsl["head.w"], np.tensordot(act["b5"], dyn, axes=([0, 1, 2], [0, 1, 2])))
    cmp("head.b", gsl["head.b"], np.array([dyn.sum()]))
    cmp("d b5", grad["b5"], bf16_round(dyn[..., None] * p["head.w"]) * (act["b5"] > 0))

    def layer(name, x, dout, mask=None):
        """parameter gradients of layer `name` from its stored input x and
        stored (masked) output gradient; returns its BF16 input gradient,
        masked by `mask` > 0 when given."""
        dx, dw, db = U.conv3_backward(x, pb[name + ".w"], dout)
        cmp(name + ".w", gsl[name + ".w"], dw)
        cmp(name + ".b", gsl[name + ".b"], db)
        dx = bf16_round(dx)
        return dx * (mask > 0) if mask is not None else dx

    cmp("d a5", grad["a5"], layer("l5b", act["a5"], grad["b5"], act["a5"]))
    dc1 = layer("l5a", act["c1"], grad["a5"])
    cmp("d c1[up]", grad["c1"][..., :32], dc1[..., :32])
    cmp("d b4", grad["b4"], bf16_round(U.up_backward(grad["c1"][..., :32])) * (act["b4"] > 0))
    cmp("d a4", grad["a4"], layer("l4b", act["a4"], grad["b4"], act["a4"]))
    dc2 = layer("l4a", act["c2"], grad["a4"])
    cmp("d c2[up]", grad["c2"][..., :64], dc2[..., :64])
    cmp("d b3", grad["b3"], bf16_round(U.up_backward(grad["c2"][..., :64])) * (act["b3"] > 0))
    cmp("d a3", grad["a3"], layer("l3b", act["a3"], grad["b3"], act["a3"]))
    cmp("d p2", grad["p2"], layer("l3a", act["p2"], grad["a3"]))
    s2 = act["c2"][..., 64:]
    cmp("d s2", grad["c2"][..., 64:], bf16_round(dc2[..., 64:] + U.pool_backward(grad["p2"])) * (s2 > 0))
    cmp("d a2", grad["a2"], layer("l2b", act["a2"], grad["c2"][..., 64:], act["a2"]))
    cmp("d p1", grad["p1"], layer("l2a", act["p1"], grad["a2"]))
    s1 = act["c1"][..., 32:]
    cmp("d s1", grad["c1"][..., 32:], bf16_round(dc1[..., 32:] + U.pool_backward(grad["p1"])) * (s1 > 0))
    cmp("d a1", grad["a1"], layer("l1b", act["a1"], grad["c1"][..., 32:], act["a1"]))
    layer("l1a", act["x0"], grad["a1"])
    wkeys = [k for k in errs if not k.startswith("d ")]
    dkeys = [k for k in errs if k.startswith("d ")]
    print("backward stages: max parameter-gradient error %.2e (%s), max activation-gradient error %.2e (%s)" % (
        max(errs[k] for k in wkeys), max(wkeys, key=errs.get), max(errs[k] for k in dkeys), max(dkeys, key=errs.get)))
    assert all(errs[k] < 1e-5 for k in wkeys), {k: errs[k] for k in wkeys}
    assert all(errs[k] < 1e-4 for k in dkeys), {k: errs[k] for k in dkeys}
    # deterministic: a second backward gives the same bits
    grads2 = torch.zeros_like(grads)
    net.backward(torch.from_numpy(dy).cuda(), n, grads2)
    assert torch.equal(grads, grads2)


def test_train_step_is_forward_backward_adam(P):
    """ws_unet_train_step equals its composition: the training forward pass,
    dL/dyhat = 2 (yhat - t) / n^3 for the MSE loss against the solved field's
    source target, ws_unet_backward and ws_adam_step."""
    import oracle
    from paper_2604_15434_amd.warmstart import WarmStart, adam_step

    n = 64
    rho, prm = _net_case(n, seed=6)
    c = oracle.eft_coefficients(**prm)
    chi = _smooth_chi(n)
    t = U.source_target(chi, rho, c["s"] * c["mu_chi"]).astype(np.float32).reshape(-1)
    rho_d, chi_d = torch.from_numpy(rho).cuda(), torch.from_numpy(chi).cuda()
    a = WarmStart(seed=4)
    b = WarmStart(seed=4)
    ga = torch.zeros(a.params.numel(), dtype=torch.float32, device="cuda")
    a.train_step(rho_d, chi_d, prm, 1e-3, grad_clip=0.5, grad_out=ga)
    yhat = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    b.forward_train(rho_d, prm, yhat)
    dy = torch.from_numpy((2.0 / n**3) * (yhat.cpu().numpy() - t)).float().cuda()
    gb = torch.zeros_like(ga)
    b.backward(dy, n, gb)
    assert rel(gb.cpu().numpy().astype(np.float64), ga.cpu().numpy().astype(np.float64)) < 1e-4
    adam_step(b.params, ga, b.m, b.v, 1, 1e-3, grad_clip=0.5)
    assert torch.equal(a.params, b.params) and torch.equal(a.m, b.m) and torch.equal(a.v, b.v)


def test_adam_step_matches_oracle(P):
    """ws_adam_step against the oracle's Adam, element by element, over three
    steps (the second with global-norm clipping active), from FP32 state:
    parameters and moments within 1e-6 relative."""
    from paper_2604_15434_amd.warmstart import adam_step

    rng = np.random.default_rng(8)
    nprm = 100_003
    w = rng.standard_normal(nprm).astype(np.float32)
    m = np.zeros(nprm, dtype=np.float32)
    v = np.zeros(nprm, dtype=np.float32)
    wd, md, vd = (torch.from_numpy(x.copy()).cuda() for x in (w, m, v))
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    for step, clip in ((1, 0.0), (2, 5.0), (3, 1e6)):
        g = (rng.standard_normal(nprm) * 10.0 ** rng.uniform(-4, 1, nprm)).astype(np.float32)
        w_in, m_in, v_in = (t.cpu().numpy().astype(np.float64) for t in (wd, md, vd))
        gn = adam_step(wd, torch.from_numpy(g).cuda(), md, vd, step, lr, b1, b2, eps, grad_clip=clip, want_norm=True)
        w_ref, m_ref, v_ref, gn_ref = U.adam_step(w_in, g.astype(np.float64), m_in, v_in, step, lr, b1, b2, eps,
                                                  grad_clip=clip)
        assert gn == pytest.approx(gn_ref, rel=1e-12)
        if step == 2:
            assert gn_ref > clip  # clipping is active in this step
        gc = g.astype(np.float64) * (min(1.0, clip / gn_ref) if clip > 0 else 1.0)
        # FP32 arithmetic: each result within 1e-6 of the magnitudes it is formed from
        scales = ((wd, w_ref, np.abs(w_in) + np.abs(w_ref - w_in)),
                  (md, m_ref, b1 * np.abs(m_in) + (1 - b1) * np.abs(gc)),
                  (vd, v_ref, b2 * np.abs(v_in) + (1 - b2) * gc * gc))
        for got, ref, scale in scales:
            gg = got.cpu().numpy().astype(np.float64)
            bad = np.abs(gg - ref) > 1e-6 * scale + 1e-30
            assert not bad.any(), (step, int(bad.sum()), float(np.max(np.abs(gg - ref) / (scale + 1e-300))))
        # the update itself, where it is not lost in w's own rounding
        upd, upd_ref = w_in - wd.cpu().numpy().astype(np.float64), w_in - w_ref
        big = np.abs(upd_ref) > 1e-3 * np.abs(w_in)
        np.testing.assert_allclose(upd[big], upd_ref[big], rtol=2e-4)


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_learned_guess_reaches_the_same_field(P, precision):
    """Whatever the network predicts, the solve from the learned guess
    converges to the field of the zero-guess solve (the guess changes the
    cost, not the answer)."""
    from paper_2604_15434_amd.warmstart import WarmStart
    from workloads import lognormal_density

    n = 64
    rho = torch.from_numpy(lognormal_density(n, 125.0, seed=9)).cuda()
    prm = dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.05, a=0.9)
    net = WarmStart(seed=1)
    tol = 1e-11 if precision == "f64" else 1e-9
    chi_ref = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    P.mg_scalar_solve(rho, prm, P.MgOpts(rel_tol=tol, max_vcycles=60, precision=precision), chi_ref)
    chi = torch.zeros_like(chi_ref)
    rep = P.mg_scalar_solve(rho, prm, P.MgOpts(rel_tol=tol, max_vcycles=60, precision=precision, guess="learned",
                                               learned=net), chi)
    assert rep["status"] == 0 and rep["rel_residual"] <= tol
    err = float((chi - chi_ref).norm() / chi_ref.norm())
    assert err < 1e-8, err


def test_learned_guess_rejects_bad_grid(P):
    from paper_2604_15434_amd.warmstart import WarmStart
    from workloads import lognormal_density

    rho = torch.from_numpy(lognormal_density(48, 94.0, seed=9)).cuda()
    net = WarmStart(seed=1)
    chi = torch.zeros_like(rho)
    with pytest.raises(P.PmError):
        P.mg_scalar_solve(rho, dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=1.0),
                          P.MgOpts(guess="learned", learned=net), chi)


def test_trained_network_gain_on_held_out_fields(P):
    """What the trained network (committed weights) gains over the method
    without it, on deposited 128^3 lognormal particle loads of seeds outside
    the training range and fresh parameter draws: its source error is far below the untrained
    network's, the solve from its guess starts from a smaller residual than
    the zero-guess full multigrid and never needs more V-cycles, and the
    final field is the zero-guess one.  (Wall time is reported, not asserted:
    the network's pass costs about as much as the cycle it saves.)"""
    import os

    from paper_2604_15434_amd.warmstart import DEFAULT_WEIGHTS, WarmStart
    from workloads import lognormal_particles, scan_params

    if not os.path.exists(DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    net = WarmStart.load(DEFAULT_WEIGHTS)
    untrained = WarmStart(seed=0)
    n = 128
    prms = scan_params(4, seed=5000)
    for k, prm in enumerate(prms):
        pos, _ = lognormal_particles(n, 250.0, seed=5000 + k)
        rho = torch.empty((n, n, n), dtype=torch.float64, device="cuda")
        P.pm_deposit(torch.from_numpy(pos).cuda(), n, rho)
        ref = torch.zeros_like(rho)
        P.mg_scalar_solve(rho, prm, P.MgOpts(rel_tol=1e-10, max_vcycles=80), ref)
        e_tr = math.sqrt(net.train_step(rho, ref, prm, 0.0)) / float(rho.std())
        e_un = math.sqrt(untrained.train_step(rho, ref, prm, 0.0)) / float(rho.std())
        out = {}
        for g in ("zero", "learned"):
            chi = torch.zeros_like(rho)
            rep = P.mg_scalar_solve(rho, prm, P.MgOpts(rel_tol=1e-7, max_vcycles=60, precision="mixed", guess=g,
                                                       learned=net), chi)
            assert rep["status"] == 0
            out[g] = (chi, rep)
        z, l = out["zero"][1], out["learned"][1]
        print(f"seed {5000 + k}: source error {e_tr:.3f} (untrained {e_un:.3f}); first residual "
              f"{l['residual_hist'][0]:.2e} vs {z['residual_hist'][0]:.2e}; V-cycles {l['vcycles']} vs "
              f"{z['vcycles']}; ms {l['ms']:.2f} vs {z['ms']:.2f}")
        assert e_tr < 0.2 and e_tr < 0.5 * e_un
        assert l["residual_hist"][0] < 0.5 * z["residual_hist"][0]
        assert l["vcycles"] <= z["vcycles"]
        err = float((out["learned"][0] - ref).norm() / ref.norm())
        assert err < 1e-5


def test_step_overlaps_network_and_keeps_the_field(P):
    """pm_step runs the warm start's network, the warm-start pass and the
    scalar solve on a second stream, beside the Poisson solve.  The step must
    give the fields of the zero-guess step (to the solve tolerance), the same
    psi, and be deterministic from run to run."""
    from paper_2604_15434_amd.warmstart import DEFAULT_WEIGHTS, WarmStart
    from workloads import lognormal_particles

    ng = 64
    pos_np, _ = lognormal_particles(ng, 125.0, seed=31)
    prm = dict(omega_m0=0.3071, alpha_b0=-0.5, alpha_m0=0.05, a=0.8)
    net = WarmStart.load(DEFAULT_WEIGHTS)
    out = {}
    for tag, guess in (("zero", "zero"), ("learned", "learned"), ("learned2", "learned")):
        pos = torch.from_numpy(pos_np).cuda()
        vel = torch.zeros_like(pos)
        psi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
        chi = torch.zeros_like(psi)
        po = P.MgOpts(rel_tol=1e-11, max_vcycles=60, precision="mixed")
        so = P.MgOpts(rel_tol=1e-11, max_vcycles=60, precision="mixed", guess=guess,
                      learned=net if guess == "learned" else None)
        rep = P.pm_step(pos, vel, ng, prm, po, so, 1e-2, 0.0, psi, chi)
        assert rep["status"] == 0, rep
        torch.cuda.synchronize()
        out[tag] = (psi.clone(), chi.clone(), vel.clone())
    for i in range(3):
        a, b = out["learned"][i], out["learned2"][i]
        assert torch.equal(a, b), i
    err_chi = float((out["learned"][1] - out["zero"][1]).norm() / out["zero"][1].norm())
    err_v = float((out["learned"][2] - out["zero"][2]).norm() / out["zero"][2].norm())
    assert err_chi < 1e-8 and err_v < 1e-8, (err_chi, err_v)
    assert torch.equal(out["learned"][0], out["zero"][0])


@pytest.mark.parametrize("cin,cout", [(48, 16), (96, 32)])
def test_upsampled_layer_polyphase_matches_reference(P, cin, cout):
    """Inference form of a decoder layer whose input is [upsampled coarse
    tensor | skip tensor]: the polyphase convolution of the coarse tensor plus
    the convolution of the skip channels equals the convolution of the
    concatenation (oracle, FP64, BF16-rounded operands).  The polyphase
    weights are sums of up to 8 taps rounded once to BF16, so the bound is
    that of BF16 weights (1e-2 relative), not the FP32-accumulation one."""
    n = 128
    up, sub = 2 * cin // 3, cin // 3
    rng = np.random.default_rng(cin)
    xc = rng.standard_normal((n // 2, n // 2, n // 2, up))
    xs = rng.standard_normal((n, n, n, sub))
    w = rng.standard_normal((27, cin, cout)) * 0.05
    b = rng.standard_normal(cout)
    L = P._lib
    out = torch.zeros(n**3 * cout, dtype=torch.float32, device="cuda")
    wb = (54 * cin * ((cout + 15) // 16 * 16) + 255) // 256 * 256
    wsz = 2 * wb + 4 * 240 * (27 * cin * cout + cout)
    ws = torch.empty(wsz, dtype=torch.uint8, device="cuda")
    wd = torch.from_numpy(w.astype(np.float32)).cuda()
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    xcd, xsd = dev_bits(bf16_bits(xc)), dev_bits(bf16_bits(xs))
    ptr = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    rc = L.lib().ws_conv3(3, n, cin, cout, ptr(xcd), ptr(xsd), ptr(wd), ptr(bd), ptr(out), ptr(ws), wsz,
                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    got = out.cpu().numpy().astype(np.float64).reshape(n, n, n, cout)
    # reference at 4096 sampled voxels: the 27 taps of the concatenated input,
    # the upsampled channels read from the coarse parent of each neighbour
    v = rng.integers(0, n, size=(4096, 3))
    xcr, xsr, wr = bf16_round(xc), bf16_round(xs), bf16_round(w)
    ref = np.tile(b.astype(np.float32).astype(np.float64), (len(v), 1))
    for t, d in enumerate(U.TAPS):
        q = (v + np.asarray(d)) % n
        xin = np.concatenate([xcr[q[:, 0] // 2, q[:, 1] // 2, q[:, 2] // 2], xsr[q[:, 0], q[:, 1], q[:, 2]]], axis=1)
        ref += xin @ wr[t]
    g = got[v[:, 0], v[:, 1], v[:, 2]]
    err = rel(g, ref)
    print(f"polyphase layer cin {cin} cout {cout}: rel err {err:.2e}")
    assert err < 1e-2, err


@pytest.mark.parametrize("n", [64, 128])
def test_first_layer_inference_form_matches_reference(P, n):
    """Inference form of the first layer: the single-channel convolution of
    the density feature plus the broadcast channels folded into the bias
    equals the 4-channel convolution of [f, x1, x2, x3] (oracle, FP64,
    BF16-rounded operands; FP32 accumulation only: 1e-5)."""
    rng = np.random.default_rng(n + 1)
    f = rng.standard_normal((n, n, n))
    w = rng.standard_normal((27, 4, 16)) * 0.1
    b = rng.standard_normal(16)
    xc = np.array([-0.55, 0.13, 0.71], dtype=np.float32)
    fd = dev_bits(bf16_bits(f))
    wd = torch.from_numpy(w.astype(np.float32)).cuda()
    bd = torch.from_numpy(b.astype(np.float32)).cuda()
    out = torch.zeros(n**3 * 16, dtype=torch.float32, device="cuda")
    xcc = (ctypes.c_float * 3)(*xc.tolist())
    rc = P._lib.lib().ws_conv3_first(n, ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(wd.data_ptr()),
                                     ctypes.c_void_p(bd.data_ptr()), xcc, ctypes.c_void_p(out.data_ptr()),
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0
    got = out.cpu().numpy().astype(np.float64).reshape(n, n, n, 16)
    x4 = np.empty((n, n, n, 4))
    x4[..., 0] = bf16_round(f)
    x4[..., 1:] = bf16_round(xc)
    ref = U.conv3(x4, bf16_round(w), b.astype(np.float32).astype(np.float64))
    assert rel(got, ref) < 1e-5


@pytest.mark.parametrize("n", [64, 128])
def test_last_layer_with_head_matches_reference(P, n):
    """Inference form of the last layer: the 16 -> 16 convolution with ReLU
    and the 1x1x1 head applied in its epilogue, yhat = hb + sum_o hw[o]
    relu(conv(x)[o]), against the oracle on the same BF16-rounded operands
    (FP32 accumulation only: 1e-5)."""
    rng = np.random.default_rng(3 * n)
    x = rng.standard_normal((n, n, n, 16))
    w = rng.standard_normal((27, 16, 16)) * 0.1
    b = rng.standard_normal(16) * 0.1
    hw = rng.standard_normal(16) * 0.25
    hb = np.array([0.03])
    got = _conv(P, 4, n, 16, 16, x=x, w=w, b=np.concatenate([b, hw, hb])).reshape(n, n, n)
    h = U.relu(U.conv3(bf16_round(x), bf16_round(w), b.astype(np.float32).astype(np.float64)))
    ref = h @ hw.astype(np.float32).astype(np.float64) + float(np.float32(hb[0]))
    assert rel(got, ref) < 1e-5


@pytest.mark.parametrize("n", [128, 256])
def test_inference_forward_matches_oracle_samples(P, n):
    """The whole network as inference runs it (first layer on the density
    channel, polyphase decoder layers with compact skip tensors -- the first
    decoder layer only from 256^3 -- and the head in the last layer's
    epilogue) against the FP64 oracle network at sampled voxels stored by
    tests/golden/make_unet_forward.py (BF16 activations between layers:
    3e-2, as for the whole-network test)."""
    import importlib.util
    import os

    from paper_2604_15434_amd.warmstart import WarmStart

    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("make_unet_forward", os.path.join(here, "make_unet_forward.py"))
    G = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(G)
    rows = np.loadtxt(os.path.join(here, f"unet_forward_{n}.txt"), comments="#")
    idx, ref = rows[:, 0].astype(np.int64), rows[:, 1]
    assert np.array_equal(idx, G.sample_index(n))
    net = WarmStart(params=G.flat_params())
    rho = torch.from_numpy(G.density(n)).cuda()
    yhat = torch.zeros(n**3, dtype=torch.float32, device="cuda")
    net.predict(rho, dict(omega_m0=0.3071, **G.PARAMS), yhat)
    got = yhat.cpu().numpy().astype(np.float64)[idx]
    assert rel(got, ref) < 3e-2, rel(got, ref)


def test_learned_guess_entry_is_the_solves_starting_field(P):
    """ws_unet_guess returns chi_0, the field a solve with guess "learned"
    starts from: a solve from it (guess "given") starts at the learned
    solve's first residual, takes as many V-cycles and reaches the same
    field; chi_0 is mean-free."""
    from paper_2604_15434_amd.warmstart import DEFAULT_WEIGHTS, WarmStart
    from workloads import lognormal_density

    import os

    if not os.path.exists(DEFAULT_WEIGHTS):
        pytest.skip("no trained weights")
    net = WarmStart.load(DEFAULT_WEIGHTS)
    n = 64
    rho = torch.from_numpy(lognormal_density(n, 125.0, seed=31)).cuda()
    prm = dict(omega_m0=0.3071, alpha_b0=-0.5, alpha_m0=0.1, a=0.9)
    chi0 = torch.zeros_like(rho)
    net.guess(rho, prm, chi0)
    assert abs(float(chi0.mean())) < 1e-12 * float(chi0.abs().max())
    opts = dict(rel_tol=1e-10, max_vcycles=60)
    chi_l = torch.zeros_like(rho)
    rl = P.mg_scalar_solve(rho, prm, P.MgOpts(guess="learned", learned=net, **opts), chi_l)
    chi_g = chi0.clone()
    rg = P.mg_scalar_solve(rho, prm, P.MgOpts(guess="given", **opts), chi_g)
    assert rl["status"] == rg["status"] == 0
    assert rg["residual_hist"][0] == pytest.approx(rl["residual_hist"][0], rel=1e-6)
    assert abs(rl["vcycles"] - rg["vcycles"]) <= 1
    assert float((chi_g - chi_l).norm() / chi_l.norm()) < 1e-8
