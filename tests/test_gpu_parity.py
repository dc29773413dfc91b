"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Tolerances: relative scalar-field error 1e-10 (FP64
path, both sides solved to relative residual 1e-12) and 1e-5 (mixed
precision at 1e-7), force RMS error 1e-4 relative."""
import numpy as np
import pytest

import oracle
from workloads import config_params, lattice_displacement_ics, lognormal_density, lognormal_particles

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_2604_15434_amd as P

    return P


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _mean_free(x):
    x = np.asarray(x, dtype=np.float64)
    return x - x.mean()


CFG0 = config_params("cfg0")[0]


# ------------------------------------------------------------------ deposit
@pytest.mark.parametrize("ng,kind", [(32, "lattice"), (64, "lognormal"), (24, "lattice"), (128, "lognormal")])
def test_deposit_matches_oracle(P, ng, kind):
    """CIC deposit against the oracle; a permuted particle list gives bitwise
    the same grid (fixed-point sums).  At 128^3 each block walks several
    1024-particle chunks."""
    if kind == "lattice":
        pos = lattice_displacement_ics(ng, 100.0, seed=0)
    else:
        pos, _ = lognormal_particles(ng, 500.0 * ng / 256, seed=2)
    ref = oracle.cic_deposit(pos, ng)
    rho = torch.empty((ng, ng, ng), dtype=torch.float64, device="cuda")
    P.pm_deposit(dev(pos), ng, rho)
    got = rho.cpu().numpy()
    assert np.abs(got - ref).max() < 1e-10
    # order independence: a permuted particle list gives bitwise the same grid
    perm = np.random.default_rng(0).permutation(pos.shape[1])
    rho2 = torch.empty_like(rho)
    P.pm_deposit(dev(pos[:, perm]), ng, rho2)
    assert torch.equal(rho, rho2)
    rho32 = torch.empty((ng, ng, ng), dtype=torch.float32, device="cuda")
    P.pm_deposit(dev(pos, torch.float32), ng, rho32)
    assert np.abs(rho32.cpu().numpy() - ref).max() < 2e-5 * max(1.0, ref.max())


@pytest.mark.parametrize("ng,dtype", [(32, torch.float64), (64, torch.float32), (128, torch.float64),
                                      (128, torch.float32)])
def test_sorted_deposit_gathers_the_same_grid(P, ng, dtype):
    """Particles in CIC base-row order (pm_sort_particles) take the gather
    deposit (every cell summed once, no global atomics); the grid is bitwise
    the scatter's (the same 2^-40 integer sums) and matches the oracle.  One
    pair of particles swapped out of order sends the deposit back to the
    scatter, again bitwise the same."""
    pos_np, _ = lognormal_particles(ng, 500.0 * ng / 256, seed=12)
    pos = torch.from_numpy(pos_np).to("cuda", dtype)
    rho_scatter = torch.empty((ng, ng, ng), dtype=dtype, device="cuda")
    P.pm_deposit(pos, ng, rho_scatter)  # lognormal loads are in cell order, not base-row order: scatter
    P.pm_sort_particles(pos, ng)
    rho_gather = torch.empty_like(rho_scatter)
    P.pm_deposit(pos, ng, rho_gather)
    assert torch.equal(rho_gather, rho_scatter)
    ref = oracle.cic_deposit(pos.cpu().numpy().astype(np.float64), ng)
    tol = 1e-10 if dtype == torch.float64 else 2e-5 * max(1.0, ref.max())
    assert np.abs(rho_gather.cpu().numpy() - ref).max() < tol
    swapped = pos.clone()
    swapped[:, [10, pos.shape[1] - 10]] = swapped[:, [pos.shape[1] - 10, 10]]
    rho_swapped = torch.empty_like(rho_scatter)
    P.pm_deposit(swapped, ng, rho_swapped)
    assert torch.equal(rho_swapped, rho_scatter)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_sorted_deposit_skips_unusable_z_like_the_scatter(P, dtype):
    """Base-row order depends on x and y only, so sorted particles whose z is
    NaN or infinite still take the gather; the gather skips them as the
    scatter does, and both grids equal the oracle's deposit of the other
    particles (normalised by the full particle count)."""
    ng = 32
    pos_np, _ = lognormal_particles(ng, 500.0 * ng / 256, seed=5)
    pos = torch.from_numpy(pos_np).to("cuda", dtype)
    P.pm_sort_particles(pos, ng)
    bad = [7, 1000, pos.shape[1] - 3]
    pos[2, bad[0]] = float("nan")
    pos[2, bad[1]] = float("inf")
    pos[2, bad[2]] = -float("inf")
    rho_gather = torch.empty((ng, ng, ng), dtype=dtype, device="cuda")
    P.pm_deposit(pos, ng, rho_gather)
    swapped = pos.clone()
    swapped[:, [10, pos.shape[1] - 10]] = swapped[:, [pos.shape[1] - 10, 10]]
    rho_scatter = torch.empty_like(rho_gather)
    P.pm_deposit(swapped, ng, rho_scatter)
    assert torch.equal(rho_gather, rho_scatter)
    keep = np.ones(pos.shape[1], dtype=bool)
    keep[bad] = False
    host = pos.cpu().numpy().astype(np.float64)
    ref = oracle.cic_deposit(host[:, keep], ng) * (keep.sum() / keep.size)
    tol = 1e-10 if dtype == torch.float64 else 2e-5 * max(1.0, ref.max())
    assert np.abs(rho_gather.cpu().numpy() - ref).max() < tol


# ------------------------------------------------------------------ Poisson
@pytest.mark.parametrize("ng", [32, 48])
def test_poisson_matches_fft_solution(P, ng):
    pos = lattice_displacement_ics(ng, 100.0, seed=0, rms_cells=0.6)
    rho = oracle.cic_deposit(pos, ng)
    c = oracle.eft_coefficients(**CFG0)
    ref = oracle.solve_poisson(oracle.density_contrast(rho), c, 1.0 / ng)
    psi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_poisson_solve(dev(rho), CFG0, P.MgOpts(rel_tol=1e-12, max_vcycles=60), psi)
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-12
    assert rel(_mean_free(psi.cpu().numpy()), ref) < 1e-10


# ------------------------------------------------------------------ scalar field
def _scalar_case(ng, kind, ab0, am0=0.0, a=1.0):
    if kind == "cfg0":
        rho = oracle.cic_deposit(lattice_displacement_ics(ng, 100.0, seed=0), ng)
        p = dict(CFG0)
    else:
        rho = lognormal_density(ng, 500.0 * ng / 256, seed=2)
        p = dict(omega_m0=0.3071, alpha_b0=ab0, alpha_m0=am0, a=a)
    return rho, p


@pytest.mark.parametrize("ng,kind,ab0,am0,a", [
    (32, "cfg0", -0.4, 0.0, 0.5),
    (32, "lognormal", -0.2, 0.0, 1.0),
    (32, "lognormal", -0.6, 0.1, 1.0),
    (64, "lognormal", -0.6, 0.0, 1.0),
])
def test_scalar_f64_matches_oracle(P, ng, kind, ab0, am0, a):
    rho, p = _scalar_case(ng, kind, ab0, am0, a)
    c = oracle.eft_coefficients(**p)
    delta = oracle.density_contrast(rho)
    ref, orep = oracle.solve_chi(delta, c, 1.0 / ng, tol=1e-12, max_cycles=200)
    assert orep["status"] == 0
    chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-12, max_vcycles=80), chi)
    assert rep["status"] == 0, rep
    assert rep["clamped_cells"] == orep["clamped"]
    got = chi.cpu().numpy()
    assert rel(_mean_free(got), ref) < 1e-10
    # the GPU solution satisfies the oracle's discrete system
    assert oracle.relative_residual(got, delta, c, 1.0 / ng) < 1e-11


def test_scalar_screening_off_matches_fft(P):
    ng = 32
    rho, _ = _scalar_case(ng, "cfg0", -0.4)
    p = dict(CFG0, screening=0)
    c = oracle.eft_coefficients(**p)
    ref = oracle.solve_chi_linear(oracle.density_contrast(rho), c, 1.0 / ng)
    chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-12, max_vcycles=60), chi)
    assert rep["status"] == 0 and rep["clamped_cells"] == 0
    assert rel(_mean_free(chi.cpu().numpy()), ref) < 1e-10


@pytest.mark.parametrize("ab0", [-0.2, -0.6])
def test_scalar_mixed_precision(P, ab0):
    ng = 64
    rho, p = _scalar_case(ng, "lognormal", ab0)
    c = oracle.eft_coefficients(**p)
    delta = oracle.density_contrast(rho)
    ref, _ = oracle.solve_chi(delta, c, 1.0 / ng, tol=1e-12, max_cycles=200)
    chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-7, max_vcycles=60, precision="mixed"), chi)
    assert rep["status"] == 0 and rep["rel_residual"] <= 1e-7, rep
    got = chi.cpu().numpy()
    assert rel(_mean_free(got), ref) < 1e-5
    assert oracle.relative_residual(got, delta, c, 1.0 / ng) < 2e-7
    # FP32 in/out arrays on the same path
    chi32 = torch.zeros((ng, ng, ng), dtype=torch.float32, device="cuda")
    rep32 = P.mg_scalar_solve(dev(rho, torch.float32), p,
                              P.MgOpts(rel_tol=1e-7, max_vcycles=60, precision="mixed"), chi32)
    assert rep32["status"] == 0
    assert rel(_mean_free(chi32.cpu().numpy()), ref) < 1e-5


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_jacobi_smoother_reaches_the_oracle_field(P, precision):
    """The pointwise local solve under-relaxed as chi <- 0.6 chi* + 0.4 chi
    (the smoother of PySCo, Secs. 3.2.1 and 3.5.1) in every level of the
    V-cycle converges to the same discrete field as the red-black
    Gauss-Seidel smoother and the oracle: the clamp-heavy 64^3 lognormal
    case; V-cycle counts of the two smoothers reported."""
    ng = 64
    rho, p = _scalar_case(ng, "lognormal", -0.6)
    c = oracle.eft_coefficients(**p)
    delta = oracle.density_contrast(rho)
    ref, orep = oracle.solve_chi(delta, c, 1.0 / ng, tol=1e-12, max_cycles=200)
    tol = 1e-12 if precision == "f64" else 1e-7
    out = {}
    for sm in ("jacobi", "rbgs"):
        chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
        rep = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=tol, max_vcycles=200, n_pre=2, n_post=2,
                                                      precision=precision, smoother=sm), chi)
        assert rep["status"] == 0, (sm, rep["rel_residual"])
        assert rep["clamped_cells"] == orep["clamped"]
        out[sm] = (_mean_free(chi.cpu().numpy()), rep["vcycles"])
    print(f"smoothers {precision}: V-cycles jacobi {out['jacobi'][1]}, red-black {out['rbgs'][1]}")
    bound = 1e-10 if precision == "f64" else 1e-5
    assert rel(out["jacobi"][0], ref) < bound
    assert rel(out["jacobi"][0], out["rbgs"][0]) < bound


def test_scalar_guesses_reach_same_solution(P):
    ng = 32
    rho, p = _scalar_case(ng, "lognormal", -0.6)
    base = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    r0 = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-11, max_vcycles=80), base)
    lin = torch.zeros_like(base)
    r1 = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-11, max_vcycles=80, guess="linear"), lin)
    given = base.clone()
    r2 = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=1e-11, max_vcycles=80, guess="given"), given)
    assert r0["status"] == r1["status"] == r2["status"] == 0
    assert r2["vcycles"] == 0
    b = base.cpu().numpy()
    assert rel(lin.cpu().numpy(), b) < 1e-9
    assert rel(given.cpu().numpy(), b) < 1e-9


# ------------------------------------------------------------------ full step
@pytest.mark.parametrize("dtype,prec,ftol", [(torch.float64, "f64", 1e-9), (torch.float32, "mixed", 1e-4)])
def test_pm_step_cfg0_matches_oracle(P, dtype, prec, ftol):
    ng = 32
    pos = lattice_displacement_ics(ng, 100.0, seed=0)
    vel = np.zeros_like(pos)
    ref = oracle.pm_step(pos, vel, ng, CFG0, dt_kick=1.0, tol=1e-12)
    tol = 1e-12 if prec == "f64" else 1e-7
    gp, gv = dev(pos, dtype), dev(vel, dtype)
    psi = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
    chi = torch.zeros_like(psi)
    rep = P.pm_step(gp, gv, ng, CFG0, P.MgOpts(rel_tol=tol, max_vcycles=80, precision=prec),
                    P.MgOpts(rel_tol=tol, max_vcycles=80, precision=prec), 1.0, 0.0, psi, chi)
    assert rep["status"] == 0, rep
    acc = gv.cpu().numpy().astype(np.float64)
    err = np.sqrt(np.mean(np.sum((acc - ref["acc"]) ** 2, 0)) / np.mean(np.sum(ref["acc"] ** 2, 0)))
    assert err < ftol
    assert rel(_mean_free(chi.cpu().numpy()), ref["chi"]) < (1e-10 if prec == "f64" else 1e-5)
    assert np.array_equal(gp.cpu().numpy(), pos.astype(gp.cpu().numpy().dtype))  # no drift requested


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_pm_step_solves_match_standalone_solves(P, prec):
    """pm_step runs its two solves side by side: the scalar field on a second
    stream from a worker thread, in a workspace region of its own.  Its fields
    must be those of the standalone solves on the step's own deposit, and
    repeated steps must agree bit for bit."""
    from workloads import lognormal_particles

    ng = 64
    pos_np, _ = lognormal_particles(ng, 125.0, seed=41)
    prm = dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.05, a=0.9)
    opts = P.MgOpts(rel_tol=1e-10, max_vcycles=80, precision=prec)
    pos = torch.from_numpy(pos_np).cuda()
    rho = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    P.pm_deposit(pos, ng, rho)
    psi_ref, chi_ref = torch.zeros_like(rho), torch.zeros_like(rho)
    assert P.mg_poisson_solve(rho, prm, opts, psi_ref)["status"] == 0
    assert P.mg_scalar_solve(rho, prm, opts, chi_ref)["status"] == 0
    outs = []
    for _ in range(2):
        vel = torch.zeros_like(pos)
        psi, chi = torch.zeros_like(rho), torch.zeros_like(rho)
        rep = P.pm_step(pos, vel, ng, prm, opts, opts, 1e-2, 0.0, psi, chi)
        assert rep["status"] == 0, rep
        torch.cuda.synchronize()
        outs.append((psi.clone(), chi.clone(), vel.clone()))
    for a, b in zip(*outs):
        assert torch.equal(a, b)
    psi, chi, _ = outs[0]
    assert float(chi_ref.norm()) > 0.0 and float(psi_ref.norm()) > 0.0
    assert float((psi - psi_ref).norm() / psi_ref.norm()) < 1e-8
    assert float((chi - chi_ref).norm() / chi_ref.norm()) < 1e-8


_CFG1_CACHE = {}


def _cfg1_ref(k):
    """Oracle step of the 128^3 Zel'dovich workload (250 Mpc/h, seed 1) for
    parameter set k (cached across precisions)."""
    if "pos" not in _CFG1_CACHE:
        from workloads import zeldovich_ics

        _CFG1_CACHE["pos"] = zeldovich_ics(128, 250.0, seed=1)
    if k not in _CFG1_CACHE:
        pos = _CFG1_CACHE["pos"]
        _CFG1_CACHE[k] = oracle.pm_step(pos, np.zeros_like(pos), 128, config_params("cfg1")[k], dt_kick=1.0,
                                        tol=1e-12)
    return _CFG1_CACHE["pos"], _CFG1_CACHE[k]


@pytest.mark.parametrize("prec", ["f64", "mixed"])
@pytest.mark.parametrize("k", range(8))
def test_pm_step_cfg1_matches_oracle(P, k, prec):
    """128^3 Zel'dovich step for the 8 parameter sets (alpha_B0 in {-0.2, -0.6},
    alpha_M0 in {0, 0.1}, a in {0.33, 1}): FP64 at 1e-12 and FP32 particles
    with mixed-precision solves at 1e-7, against the oracle at 1e-12.  Checks
    the force RMS error, the scalar field and its power spectrum per bin."""
    ng = 128
    pos, ref = _cfg1_ref(k)
    prm = config_params("cfg1")[k]
    dtype = torch.float64 if prec == "f64" else torch.float32
    tol = 1e-12 if prec == "f64" else 1e-7
    gp, gv = dev(pos, dtype), torch.zeros((3, pos.shape[1]), dtype=dtype, device="cuda")
    psi = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
    chi = torch.zeros_like(psi)
    opts = P.MgOpts(rel_tol=tol, max_vcycles=80, precision=prec)
    rep = P.pm_step(gp, gv, ng, prm, opts, opts, 1.0, 0.0, psi, chi)
    assert rep["status"] == 0, rep
    acc = gv.cpu().numpy().astype(np.float64)
    ferr = np.sqrt(np.mean(np.sum((acc - ref["acc"]) ** 2, 0)) / np.mean(np.sum(ref["acc"] ** 2, 0)))
    chi_g = _mean_free(chi.cpu().numpy())
    cerr = rel(chi_g, ref["chi"])
    _, pk_g, _ = oracle.power_spectrum(chi_g, 250.0)
    _, pk_r, _ = oracle.power_spectrum(ref["chi"], 250.0)
    perr = float(np.max(np.abs(pk_g / pk_r - 1.0)))
    print(f"cfg1[{k}] {prec}: force {ferr:.2e} chi {cerr:.2e} P_chi(k) max {perr:.2e} "
          f"V-cycles {rep['scalar']['vcycles']}/{rep['poisson']['vcycles']}")
    if prec == "f64":
        assert ferr < 1e-9 and cerr < 1e-10 and perr < 1e-9
    else:
        assert ferr < 1e-4 and cerr < 1e-5 and perr < 1e-4


def test_force_interp(P):
    """pm_force_interp: the 5-point gradient of Psi_N + xi chi interpolated
    to the particles and the kick, on random fields and positions."""
    ng = 16
    rng = np.random.default_rng(4)
    pos = rng.random((3, 500))
    vel = rng.standard_normal((3, 500)) * 0.01
    psi = rng.standard_normal((ng, ng, ng))
    chi = rng.standard_normal((ng, ng, ng))
    p = dict(omega_m0=0.3071, alpha_b0=-0.3, alpha_m0=0.1, a=0.8)
    c = oracle.eft_coefficients(**p)
    g = oracle.gradient5(psi + c["xi"] * chi, 1.0 / ng)
    acc_ref = oracle.cic_interpolate(g, pos)
    gv = dev(vel)
    acc = torch.zeros_like(gv)
    P.pm_force_interp(dev(psi), dev(chi), p, dev(pos), gv, 0.5, acc_out=acc)
    np.testing.assert_allclose(acc.cpu().numpy(), acc_ref, rtol=1e-11, atol=1e-11 * np.abs(acc_ref).max())
    np.testing.assert_allclose(gv.cpu().numpy(), vel + 0.5 * acc_ref, rtol=1e-11, atol=1e-12)


def _wrap_dist(a, b):
    d = np.abs(np.asarray(a, dtype=np.float64) - np.asarray(b, dtype=np.float64))
    return np.minimum(d, 1.0 - d)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_pm_step_drift_matches_oracle(P, dtype):
    """pm_step with a drift: after the kick, pos += vel dt_drift (mod 1).
    Velocities are large enough that about a tenth of the particles cross a
    face of the periodic box, and some start within 1e-6 of a face moving
    out of it; positions and velocities against the oracle step (FP64: 1e-12
    in position, FP32: within two FP32 ulps of 1)."""
    ng = 32
    pos = lattice_displacement_ics(ng, 100.0, seed=0)
    rng = np.random.default_rng(12)
    vel = rng.standard_normal(pos.shape) * 0.02
    edge = rng.choice(pos.shape[1], 200, replace=False)
    pos[0, edge[:100]] = 1.0 - 1e-7
    vel[0, edge[:100]] = np.abs(vel[0, edge[:100]])
    pos[1, edge[100:]] = 1e-7
    vel[1, edge[100:]] = -np.abs(vel[1, edge[100:]])
    if dtype == torch.float32:
        pos = pos.astype(np.float32).astype(np.float64)
        vel = vel.astype(np.float32).astype(np.float64)
    dt_kick, dt_drift = 0.5, 2.0
    ref = oracle.pm_step(pos, vel, ng, CFG0, dt_kick=dt_kick, dt_drift=dt_drift, tol=1e-12)
    moved = np.floor(pos + ref["vel"] * dt_drift) != 0
    assert moved.any(axis=0).mean() > 0.05  # the wrap is exercised
    gp, gv = dev(pos, dtype), dev(vel, dtype)
    psi = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
    chi = torch.zeros_like(psi)
    prec, tol = ("f64", 1e-12) if dtype == torch.float64 else ("mixed", 1e-7)
    opts = P.MgOpts(rel_tol=tol, max_vcycles=80, precision=prec)
    rep = P.pm_step(gp, gv, ng, CFG0, opts, opts, dt_kick, dt_drift, psi, chi)
    assert rep["status"] == 0, rep
    got_pos = gp.cpu().numpy().astype(np.float64)
    got_vel = gv.cpu().numpy().astype(np.float64)
    assert np.all((got_pos >= 0.0) & (got_pos < 1.0))
    if dtype == torch.float64:
        assert _wrap_dist(got_pos, ref["pos"]).max() < 1e-12
        np.testing.assert_allclose(got_vel, ref["vel"], rtol=1e-9, atol=1e-12)
    else:
        assert _wrap_dist(got_pos, ref["pos"]).max() < 1.2e-7
        vscale = np.abs(ref["vel"]).max()
        assert np.abs(got_vel - ref["vel"]).max() < 1e-4 * vscale


# ------------------------------------------------------------------ 256^3 headline workload
_CFG2_CACHE = {}


def _cfg2_ref(k, f32_positions=False):
    """Oracle step of the 256^3 lognormal workload (500 Mpc/h, log-sigma 1.5,
    seed 2; 256^3 particles) for parameter set k of that workload: the
    headline alpha_B0 = -0.2 and the clamp-heavy alpha_B0 = -0.6, alpha_M0 =
    0, a = 1.  Solved to 1e-12; cached for the module.  f32_positions: the
    positions rounded to FP32 first, the input the FP32 path deposits (the
    void test is a decision on delta: both sides must see the same load)."""
    if "pos" not in _CFG2_CACHE:
        _CFG2_CACHE["pos"], _ = lognormal_particles(256, 500.0, seed=2)
        _CFG2_CACHE["pos32"] = _CFG2_CACHE["pos"].astype(np.float32).astype(np.float64)
    pkey = "pos32" if f32_positions else "pos"
    key = (k, f32_positions)
    if key not in _CFG2_CACHE:
        pos = _CFG2_CACHE[pkey]
        print(f"[oracle] 256^3 step, parameter set {k}, {'FP32' if f32_positions else 'FP64'} positions: start",
              flush=True)
        ref = oracle.pm_step(pos, np.zeros_like(pos), 256, config_params("cfg2")[k], dt_kick=1.0, tol=1e-12)
        assert ref["report"]["status"] == 0
        _, pk, _ = oracle.power_spectrum(ref["chi"], 500.0)
        _CFG2_CACHE[key] = dict(acc=ref["acc"], chi=ref["chi"], pk=pk, clamped=ref["report"]["clamped"])
        print(f"[oracle] done ({ref['report']['vcycles']} FAS cycles)", flush=True)
    return _CFG2_CACHE[pkey], _CFG2_CACHE[key]


@pytest.mark.timeout(1200)
@pytest.mark.parametrize("shape", [3, 4])
@pytest.mark.parametrize("mode", ["f64", "mixed", "learned"])
@pytest.mark.parametrize("k", [0, 1])
def test_pm_step_256_matches_oracle(P, k, mode, shape):
    """The 256^3 step of the benchmark workload against the oracle, on the
    launch shapes the benchmark's tuning chooses from at this size (block
    cycle from 8^3; shape 3: largest tiles, 16 rows x 64 packed cells x 16
    planes, for the half-sweeps; shape 4: fused two-colour sweeps): FP64
    fields and particles at 1e-12 (chi within 1e-10),
    FP32 particles with mixed-precision solves at 1e-7 (chi within 1e-5),
    and the same with the learned warm start; force RMS error within 1e-4
    (FP64: 1e-9), the void-cell count equal, and the maximum P_chi(k) error
    reported.  The FP32 modes are compared with the oracle run on the same
    FP32 particle positions."""
    from paper_2604_15434_amd.warmstart import DEFAULT_WEIGHTS, WarmStart

    ng = 256
    pos, ref = _cfg2_ref(k, f32_positions=mode != "f64")
    prm = config_params("cfg2")[k]
    dtype = torch.float64 if mode == "f64" else torch.float32
    tol = 1e-12 if mode == "f64" else 1e-7
    saved = {w: P.pm_get_launch_shape(ng, w) for w in (4, 8)}
    try:
        for w in (4, 8):
            P.pm_set_launch_shape(ng, w, 8, shape)
        gp = dev(pos, dtype)
        gv = torch.zeros_like(gp)
        psi = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
        chi = torch.zeros_like(psi)
        opts = P.MgOpts(rel_tol=tol, max_vcycles=80, precision="f64" if mode == "f64" else "mixed")
        sopts = opts
        if mode == "learned":
            import os

            if not os.path.exists(DEFAULT_WEIGHTS):
                pytest.skip("no trained weights")
            sopts = P.MgOpts(rel_tol=tol, max_vcycles=80, precision="mixed", guess="learned",
                             learned=WarmStart.load(DEFAULT_WEIGHTS))
        rep = P.pm_step(gp, gv, ng, prm, opts, sopts, 1.0, 0.0, psi, chi)
    finally:
        for w, (bc, tiled) in saved.items():
            P.pm_set_launch_shape(ng, w, bc, tiled)
    assert rep["status"] == 0, rep
    acc = gv.cpu().numpy().astype(np.float64)
    ferr = float(np.sqrt(np.mean(np.sum((acc - ref["acc"]) ** 2, 0)) / np.mean(np.sum(ref["acc"] ** 2, 0))))
    chi_g = _mean_free(chi.cpu().numpy())
    cerr = rel(chi_g, ref["chi"])
    _, pk_g, _ = oracle.power_spectrum(chi_g, 500.0)
    perr = float(np.max(np.abs(pk_g / ref["pk"] - 1.0)))
    print(f"256^3 alpha_B0={prm['alpha_b0']} {mode} shape {shape}: force {ferr:.2e} chi {cerr:.2e} P_chi(k) max {perr:.2e} "
          f"V-cycles chi {rep['scalar']['vcycles']} psi {rep['poisson']['vcycles']} "
          f"clamped {rep['scalar']['clamped_cells']} (oracle {ref['clamped']})")
    assert rep["scalar"]["clamped_cells"] == ref["clamped"]
    if mode == "f64":
        assert ferr < 1e-9 and cerr < 1e-10
    else:
        assert ferr < 1e-4 and cerr < 1e-5


# ------------------------------------------------------------------ edge cases
# ---------------------------------------------------------------- edge cases
@pytest.mark.parametrize("ng", [8, 12])
@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_smallest_grids_match_oracle(P, ng, prec):
    """The shallowest hierarchies: 8^3 (the 4^3 coarsest level right below the
    finest) and 12^3 (the 6^3 coarsest solve by one workgroup); the scalar
    field against the oracle, Poisson against the exact FFT solve."""
    rho = lognormal_density(ng, 500.0 * ng / 256, seed=31)
    p = dict(omega_m0=0.3071, alpha_b0=-0.6, alpha_m0=0.1, a=1.0)
    c = oracle.eft_coefficients(**p)
    delta = oracle.density_contrast(rho)
    ref_chi, orep = oracle.solve_chi(delta, c, 1.0 / ng, tol=1e-12, max_cycles=400)
    ref_psi = oracle.solve_poisson(delta, c, 1.0 / ng)
    tol = 1e-12 if prec == "f64" else 1e-9
    chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_scalar_solve(dev(rho), p, P.MgOpts(rel_tol=tol, max_vcycles=100, precision=prec), chi)
    assert rep["status"] == 0 and rep["clamped_cells"] == orep["clamped"], rep
    assert rel(_mean_free(chi.cpu().numpy()), ref_chi) < (1e-10 if prec == "f64" else 1e-5)
    psi = torch.zeros_like(chi)
    rep = P.mg_poisson_solve(dev(rho), p, P.MgOpts(rel_tol=tol, max_vcycles=100, precision=prec), psi)
    assert rep["status"] == 0, rep
    assert rel(_mean_free(psi.cpu().numpy()), ref_psi) < (1e-10 if prec == "f64" else 1e-6)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_particles_on_faces_and_box_edges(P, dtype):
    """Particles at x = 0, on cell faces and centres and just below 1 (the
    largest position below the box length in the array's precision): the
    deposit equals the oracle's with the mass conserved, the same particles
    in base-cell order take the gather and give the same grid bit for bit, a
    single particle spreads over its 8 corners, and a step with them matches
    the oracle's forces."""
    import itertools

    ng = 16
    h = 1.0 / ng
    below_one = float(np.nextafter(np.float32(1.0), np.float32(0.0))) if dtype == torch.float32 else \
        float(np.nextafter(1.0, 0.0))
    coords = [0.0, 0.5 * h, h, 3.25 * h, 0.5, 1.0 - 0.5 * h, below_one]
    pos = np.array(list(itertools.product(coords, repeat=3)), dtype=np.float64).T.copy()
    npdt = np.float64 if dtype == torch.float64 else np.float32
    pos_t = pos.astype(npdt).astype(np.float64)  # the positions the GPU sees
    ref = oracle.cic_deposit(pos_t, ng)
    tol = 1e-10 if dtype == torch.float64 else 2e-5 * max(1.0, ref.max())
    gp = dev(pos_t, dtype)
    rho = torch.empty((ng, ng, ng), dtype=dtype, device="cuda")
    P.pm_deposit(gp, ng, rho)
    got = rho.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).max() < tol
    # total mass: exact fixed-point sums, then the output dtype's rounding per cell
    assert abs(got.sum() - ng ** 3) < (1e-9 if dtype == torch.float64 else 1e-5) * ng ** 3
    sorted_pos = gp.clone()
    P.pm_sort_particles(sorted_pos, ng)
    rho_g = torch.empty_like(rho)
    P.pm_deposit(sorted_pos, ng, rho_g)
    assert torch.equal(rho_g, rho)
    one = np.array([[0.3], [0.7], [below_one]])
    one_t = one.astype(npdt).astype(np.float64)
    rho1 = torch.empty_like(rho)
    P.pm_deposit(dev(one_t, dtype), ng, rho1)
    r1 = rho1.cpu().numpy().astype(np.float64)
    ref1 = oracle.cic_deposit(one_t, ng)
    # (weights rounded to 2^-40 and scaled by ng^3 / np = 4096: about 2e-9 per cell in FP64)
    assert np.count_nonzero(ref1) == 8 and np.abs(r1 - ref1).max() < (1e-8 if dtype == torch.float64 else 1e-1)
    assert abs(r1.sum() - ng ** 3) < 1e-6 * ng ** 3
    # a step: forces against the oracle (positions are not drifted)
    vel = np.zeros_like(pos_t)
    refs = oracle.pm_step(pos_t, vel, ng, CFG0, dt_kick=1.0, tol=1e-12)
    prec = "f64" if dtype == torch.float64 else "mixed"
    stol = 1e-12 if prec == "f64" else 1e-7
    gv = dev(vel, dtype)
    psi = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
    chi = torch.zeros_like(psi)
    rep = P.pm_step(gp, gv, ng, CFG0, P.MgOpts(rel_tol=stol, max_vcycles=80, precision=prec),
                    P.MgOpts(rel_tol=stol, max_vcycles=80, precision=prec), 1.0, 0.0, psi, chi)
    assert rep["status"] == 0, rep
    acc = gv.cpu().numpy().astype(np.float64)
    err = np.sqrt(np.mean(np.sum((acc - refs["acc"]) ** 2, 0)) / np.mean(np.sum(refs["acc"] ** 2, 0)))
    assert err < (1e-9 if dtype == torch.float64 else 1e-4)


def test_lcdm_gives_zero_scalar_field(P):
    ng = 16
    rho = lognormal_density(ng, 30.0, seed=1)
    chi = torch.ones((ng, ng, ng), dtype=torch.float64, device="cuda")
    rep = P.mg_scalar_solve(dev(rho), dict(omega_m0=0.3, alpha_b0=0.0, alpha_m0=0.0, a=1.0), P.MgOpts(), chi)
    assert rep["status"] == 0 and float(chi.abs().max()) == 0.0


def test_error_codes(P):
    ng = 16
    rho = dev(lognormal_density(ng, 30.0, seed=1))
    chi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PmError) as e:
        P.mg_scalar_solve(rho, dict(omega_m0=0.3071, alpha_b0=0.5, alpha_m0=0.0, a=1.0), P.MgOpts(), chi)
    assert e.value.code == -2
    rep = P.mg_scalar_solve(rho, dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=1.0),
                            P.MgOpts(rel_tol=1e-15, max_vcycles=1), chi)
    assert rep["status"] == -3 and rep["vcycles"] == 1
    bad = rho.clone()
    bad[3, 4, 5] = float("nan")
    with pytest.raises(P.PmError) as e:
        P.mg_scalar_solve(bad, dict(omega_m0=0.3071, alpha_b0=-0.4, alpha_m0=0.0, a=1.0), P.MgOpts(), chi)
    assert e.value.code == -4
    r10 = torch.ones((10, 10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PmError) as e:
        P.mg_poisson_solve(r10, CFG0, P.MgOpts(), torch.zeros_like(r10), ws=P.Workspace(16))
    assert e.value.code == -1
    small = P.Workspace(8)
    with pytest.raises(P.PmError) as e:
        P.mg_scalar_solve(rho, CFG0, P.MgOpts(), chi, ws=small)
    assert e.value.code == -6


def test_empty_density_gives_zero_fields(P):
    """rho = 1 everywhere (uniform lattice): delta = 0, all fields vanish."""
    ng = 16
    rho = torch.ones((ng, ng, ng), dtype=torch.float64, device="cuda")
    psi = torch.ones_like(rho)
    chi = torch.ones_like(rho)
    assert P.mg_poisson_solve(rho, CFG0, P.MgOpts(), psi)["status"] == 0
    assert P.mg_scalar_solve(rho, CFG0, P.MgOpts(), chi)["status"] == 0
    assert float(psi.abs().max()) == 0.0 and float(chi.abs().max()) == 0.0


# ---------------------------------------------------------------- batched solves
def test_batched_equals_single_solves_bitwise(P):
    """Each problem of a mixed-size batch (32^3 .. 96^3, both precisions of
    the arrays, several parameter sets) equals its own single solve bit for
    bit, and the single solves agree with the oracle."""
    import oracle
    from workloads import lognormal_density, scan_params

    sizes = [32, 48, 64, 96, 32, 64]
    prms = scan_params(len(sizes), seed=4, a=1.0)
    probs = []
    for k, (n, prm) in enumerate(zip(sizes, prms)):
        dt = torch.float64 if k % 2 == 0 else torch.float32
        rho = torch.from_numpy(lognormal_density(n, 500.0 * n / 256, seed=4000 + k)).to("cuda", dt)
        probs.append(dict(rho=rho, chi=torch.zeros_like(rho), params=prm))
    opts = P.MgOpts(rel_tol=1e-9, max_vcycles=60, precision="mixed")
    reps = P.mg_scalar_solve_batched(probs, opts)
    for k, pr in enumerate(probs):
        single = torch.zeros_like(pr["chi"])
        rep = P.mg_scalar_solve(pr["rho"], pr["params"], opts, single)
        assert torch.equal(single, pr["chi"]), k
        assert reps[k]["vcycles"] == rep["vcycles"] and reps[k]["rel_residual"] == rep["rel_residual"]
        assert reps[k]["status"] == 0
    # every member against the oracle at its own size (mixed precision at
    # 1e-9: chi within 1e-5 relative, the FP32 arrays' rounding included)
    for pr in probs:
        n = pr["rho"].shape[0]
        c = oracle.eft_coefficients(**pr["params"])
        ref, _ = oracle.solve_chi(oracle.density_contrast(pr["rho"].cpu().numpy().astype(np.float64)), c, 1.0 / n,
                                  tol=1e-12)
        got = _mean_free(pr["chi"].cpu().numpy())
        assert rel(got, ref) < 1e-5, n


def test_scan_192_members_equal_single_solves_and_the_oracle(P):
    """The 192^3 group of the parameter scan (levels down to a 6^3 coarsest
    grid): two members with the scan's parameter draws equal their single
    solves bit for bit, and the first agrees with the oracle (mixed
    precision at 1e-9: chi within 1e-5 relative)."""
    import oracle
    from workloads import lognormal_density, scan_params

    n = 192
    prms = scan_params(2, seed=9, a=1.0)
    probs = [dict(rho=torch.from_numpy(lognormal_density(n, 500.0 * n / 256, seed=4900 + k)).to("cuda", torch.float32),
                  chi=torch.zeros((n, n, n), dtype=torch.float32, device="cuda"), params=prm)
             for k, prm in enumerate(prms)]
    opts = P.MgOpts(rel_tol=1e-9, max_vcycles=60, precision="mixed")
    reps = P.mg_scalar_solve_batched(probs, opts)
    for k, pr in enumerate(probs):
        single = torch.zeros_like(pr["chi"])
        rep = P.mg_scalar_solve(pr["rho"], pr["params"], opts, single)
        assert rep["status"] == 0 and reps[k]["status"] == 0, k
        assert torch.equal(single, pr["chi"]), k
        assert reps[k]["vcycles"] == rep["vcycles"] and reps[k]["rel_residual"] == rep["rel_residual"], k
    pr = probs[0]
    c = oracle.eft_coefficients(**pr["params"])
    ref, _ = oracle.solve_chi(oracle.density_contrast(pr["rho"].cpu().numpy().astype(np.float64)), c, 1.0 / n,
                              tol=1e-10)
    err = rel(_mean_free(pr["chi"].cpu().numpy().astype(np.float64)), ref)
    print(f"scan 192^3 member vs oracle: chi rel err {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("precision,guess", [("mixed", "zero"), ("f64", "zero"), ("mixed", "linear"),
                                             ("mixed", "given")])
def test_grouped_batch_equals_single_solves_bitwise(P, precision, guess):
    """Problems of one grid and dtype are solved in lockstep, one launch per
    step for the whole group.  Members converge after different numbers of
    V-cycles (and, mixed, switch to FP64 at different outer steps), one has
    no scalar source (alpha_B0 = alpha_M0 = 0); each equals its own single
    solve bit for bit, with the same report."""
    from workloads import lognormal_density

    # (alpha_B0, alpha_M0, screening): screening off is a linear solve, run
    # as its own lockstep pass after the nonlinear members
    groups = [(48, torch.float32, [(-0.1, 0.0, 1), (-0.6, 0.1, 1), (0.0, 0.0, 1), (-0.9, 0.2, 1), (-0.3, 0.05, 1),
                                   (-0.4, 0.0, 0), (-0.8, 0.1, 0)]),
              (32, torch.float64, [(-0.2, 0.0, 1), (-1.0, 0.15, 1), (-0.5, 0.0, 1), (-0.3, 0.0, 0)])]
    probs = []
    for n, dt, pars in groups:
        for k, (ab, am, scr) in enumerate(pars):
            rho = torch.from_numpy(lognormal_density(n, 500.0 * n / 256, seed=4100 + 10 * n + k)).to("cuda", dt)
            guess0 = torch.zeros_like(rho)
            if guess == "given":
                guess0 = 1e-4 * torch.sin(torch.arange(rho.numel(), device="cuda", dtype=torch.float64)
                                          ).reshape(rho.shape).to(dt)
            probs.append(dict(rho=rho, chi=guess0.clone(), guess0=guess0,
                              params=dict(omega_m0=0.3071, alpha_b0=ab, alpha_m0=am, a=1.0, screening=scr)))
    opts = P.MgOpts(rel_tol=1e-9, max_vcycles=60, precision=precision, guess=guess)
    reps = P.mg_scalar_solve_batched(probs, opts)
    vcycles = set()
    for k, pr in enumerate(probs):
        single = pr["guess0"].clone()
        rep = P.mg_scalar_solve(pr["rho"], pr["params"], opts, single)
        assert torch.equal(single, pr["chi"]), k
        for key in ("status", "vcycles", "rel_residual", "clamped_cells", "mean_shift"):
            assert reps[k][key] == rep[key], (k, key)
        assert reps[k]["residual_hist"] == rep["residual_hist"], k
        vcycles.add(rep["vcycles"])
    assert len(vcycles) >= 3  # the members left the lockstep at different cycles
    assert float(probs[2]["chi"].abs().max()) == 0.0  # no scalar source


def test_grouped_batch_256_mixed_equals_single_solves_bitwise(P):
    """From 256^3 up the mixed solve applies each FP32 correction inside the
    next outer residual and writes the corrected FP64 iterate to the level's
    second buffer, so a member's field sits in either buffer when it leaves
    the FP32 phase (converged, or switching to FP64) and is copied back per
    slot.  Members that leave after different numbers of outer steps (and a
    linear member, screening off) each equal their own single solve bit for
    bit, with the same report."""
    from workloads import lognormal_density

    pars = [(-0.2, 0.0, 1), (-0.6, 0.1, 1), (-0.05, 0.0, 1), (-0.4, 0.0, 0)]
    probs = []
    for k, (ab, am, scr) in enumerate(pars):
        rho = torch.from_numpy(lognormal_density(256, 500.0, seed=5200 + k)).to("cuda", torch.float32)
        probs.append(dict(rho=rho, chi=torch.zeros_like(rho),
                          params=dict(omega_m0=0.3071, alpha_b0=ab, alpha_m0=am, a=1.0, screening=scr)))
    opts = P.MgOpts(rel_tol=1e-9, max_vcycles=60, precision="mixed", guess="zero")
    reps = P.mg_scalar_solve_batched(probs, opts)
    hists = set()
    for k, pr in enumerate(probs):
        single = torch.zeros_like(pr["rho"])
        rep = P.mg_scalar_solve(pr["rho"], pr["params"], opts, single)
        assert rep["status"] == 0, (k, rep["status"])
        assert torch.equal(single, pr["chi"]), k
        for key in ("status", "vcycles", "rel_residual", "clamped_cells", "mean_shift"):
            assert reps[k][key] == rep[key], (k, key)
        assert reps[k]["residual_hist"] == rep["residual_hist"], k
        hists.add(len(rep["residual_hist"]))
    assert len(hists) >= 2  # the members left the FP32 phase at different outer steps


def test_batched_rejects_learned_and_bad_sizes(P):
    rho = torch.ones((32, 32, 32), dtype=torch.float64, device="cuda")
    prm = dict(omega_m0=0.3071, alpha_b0=-0.2, alpha_m0=0.0, a=1.0)
    import ctypes

    L = P._lib
    chi = torch.zeros_like(rho)
    arr = (L.Problem * 1)(L.Problem(rho.data_ptr(), chi.data_ptr(), 32, L.PM_F64, P._params(prm)))
    o = P.MgOpts().c()
    o.guess = L.PM_GUESS_LEARNED  # rejected before any pointer is used
    o.learned_params = o.learned_ws = 256
    ws = torch.empty(P.mg_batched_workspace_bytes([dict(rho=rho, chi=chi, params=prm)]), dtype=torch.uint8,
                     device="cuda")
    rc = L.lib().mg_scalar_solve_batched(arr, 1, ctypes.byref(o), None, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                         ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.PM_EINVAL
    bad = torch.ones((7, 7, 7), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PmError):
        P.mg_scalar_solve_batched([dict(rho=bad, chi=torch.zeros_like(bad), params=prm)], P.MgOpts())


# ---------------------------------------------------------------- launch shapes
@pytest.mark.parametrize("ng,precision", [(32, "f64"), (64, "f64"), (64, "mixed"), (96, "mixed")])
def test_block_cycle_matches_per_level_launches(P, ng, precision):
    """The single-workgroup coarse cycle and the per-level launches converge
    to the same field (they differ only in the rounding of the lagged means)."""
    rho = torch.from_numpy(lognormal_density(ng, 500.0 * ng / 256, seed=21)).cuda()
    prm = dict(omega_m0=0.3071, alpha_b0=-0.5, alpha_m0=0.05, a=1.0)
    word = 4 if precision == "mixed" else 8
    opts = P.MgOpts(rel_tol=1e-11, max_vcycles=60, precision=precision)
    out = {}
    try:
        for n in (0, 16, 32):
            P.pm_set_launch_shape(ng, word, n)
            if precision == "mixed":
                P.pm_set_launch_shape(ng, 8, n)
            chi = torch.zeros_like(rho)
            rep = P.mg_scalar_solve(rho, prm, opts, chi)
            assert rep["status"] == 0, (n, rep["rel_residual"])
            out[n] = (chi, rep)
    finally:
        P.pm_set_launch_shape(ng, word, 8)
        P.pm_set_launch_shape(ng, 8, 8)
    ref = out[0][0]
    for n in (16, 32):
        err = float((out[n][0] - ref).norm() / ref.norm())
        assert err < 1e-9, (n, err)
        assert abs(out[n][1]["vcycles"] - out[0][1]["vcycles"]) <= 2
    # Poisson through the same machinery
    psi0, psi1 = torch.zeros_like(rho), torch.zeros_like(rho)
    P.pm_set_launch_shape(ng, word, 0)
    P.mg_poisson_solve(rho, prm, opts, psi0)
    P.pm_set_launch_shape(ng, word, 32)
    P.mg_poisson_solve(rho, prm, opts, psi1)
    P.pm_set_launch_shape(ng, word, 8)
    assert float((psi1 - psi0).norm() / psi0.norm()) < 1e-9


@pytest.mark.parametrize("ng,precision", [(64, "f64"), (128, "f64"), (128, "mixed"), (192, "mixed"), (256, "mixed"),
                                          (256, "f64")])
def test_tiled_smoother_matches_untiled(P, ng, precision):
    """The 2.5D-tiled half-sweep computes the same cell updates; whole solves
    differ only through the grouping of the lagged-mean partial sums.  Shape
    4 (the fused two-colour sweep on the levels of 128^3 and up whose tiles
    divide them: FP32 at 128 and 256, FP64 at 128, 192 and 256) reaches the
    same field: its black half takes the lagged mean of its red half."""
    rho = torch.from_numpy(lognormal_density(ng, 500.0 * ng / 256, seed=23)).cuda()
    prm = dict(omega_m0=0.3071, alpha_b0=-0.6, alpha_m0=0.1, a=1.0)
    opts = P.MgOpts(rel_tol=1e-11, max_vcycles=60, precision=precision)
    out = {}
    try:
        for tiled in (0, 1, 2, 3, 4):
            for word in (4, 8):
                P.pm_set_launch_shape(ng, word, 8, tiled)
            chi = torch.zeros_like(rho)
            rep = P.mg_scalar_solve(rho, prm, opts, chi)
            assert rep["status"] == 0
            out[tiled] = (chi, rep)
            if tiled == 4:  # the Poisson solve through the fused linear sweep as well
                psi4, psi0 = torch.zeros_like(rho), torch.zeros_like(rho)
                assert P.mg_poisson_solve(rho, prm, opts, psi4)["status"] == 0
                for word in (4, 8):
                    P.pm_set_launch_shape(ng, word, 8, 0)
                assert P.mg_poisson_solve(rho, prm, opts, psi0)["status"] == 0
                assert float((psi4 - psi0).norm() / psi0.norm()) < 1e-9
    finally:
        for word in (4, 8):
            P.pm_set_launch_shape(ng, word, 8, 1)
    for tiled in (1, 2, 3, 4):
        err = float((out[tiled][0] - out[0][0]).norm() / out[0][0].norm())
        assert err < 1e-9, (tiled, err)
        assert abs(out[tiled][1]["vcycles"] - out[0][1]["vcycles"]) <= 1
        assert out[tiled][1]["clamped_cells"] == out[0][1]["clamped_cells"]


def test_autotune_picks_a_candidate(P):
    ng = 64
    n, tiled = P.pm_autotune(ng, "mixed")
    assert n in (0, 8, 16, 32) and tiled in (0, 1, 2, 3, 4)
    rho = torch.from_numpy(lognormal_density(ng, 125.0, seed=22)).cuda()
    chi = torch.zeros_like(rho)
    rep = P.mg_scalar_solve(rho, dict(omega_m0=0.3071, alpha_b0=-0.3, alpha_m0=0.0, a=1.0),
                            P.MgOpts(rel_tol=1e-9, precision="mixed"), chi)
    assert rep["status"] == 0
    P.pm_set_launch_shape(ng, 4, 8, 1)


# ---------------------------------------------------------------- particle sort
@pytest.mark.parametrize("ng,npart,dtype", [(32, 50000, torch.float64), (64, 262144, torch.float32),
                                            (16, 1, torch.float64), (64, 300001, torch.float64)])
def test_sort_particles_is_stable_argsort(P, ng, npart, dtype):
    """The permutation equals NumPy's stable argsort of the CIC base-cell key
    (bit-exact), pos/vel/ids move together, and the deposit is unchanged
    (it is exact in fixed point)."""
    rng = np.random.default_rng(ng + npart)
    pos_np = rng.random((3, npart))
    pos_np[:, : npart // 3] = np.round(pos_np[:, : npart // 3] * ng) / ng  # many ties and cell edges
    pos = torch.from_numpy(pos_np).to("cuda", dtype)
    vel = torch.from_numpy(rng.standard_normal((3, npart))).to("cuda", dtype)
    ids = torch.arange(npart, dtype=torch.int64, device="cuda")
    rho0 = torch.zeros((ng, ng, ng), dtype=dtype, device="cuda")
    P.pm_deposit(pos, ng, rho0)
    p64 = pos.cpu().numpy().astype(np.float64)
    cell = np.mod(np.floor(p64 * ng - 0.5).astype(np.int64), ng)
    key = (cell[0] * ng + cell[1]) * ng + cell[2]
    order = np.argsort(key, kind="stable")
    vel0 = vel.clone()
    P.pm_sort_particles(pos, ng, vel=vel, ids=ids)
    assert np.array_equal(ids.cpu().numpy(), order)
    assert torch.equal(pos.cpu(), torch.from_numpy(p64[:, order]).to(dtype))
    assert torch.equal(vel.cpu(), vel0.cpu()[:, torch.from_numpy(order)])
    rho1 = torch.zeros_like(rho0)
    P.pm_deposit(pos, ng, rho1)
    assert torch.equal(rho0, rho1)


@pytest.mark.parametrize("prec", ["f64", "mixed"])
def test_step_on_the_callers_stream_alone_gives_the_same_bits(P, prec):
    """pm_set_step_concurrency(False): both solves issued from the calling
    thread on the caller's stream (no library thread or stream) give the
    side-by-side step's fields and velocities bit for bit."""
    ng = 64
    pos_np, _ = lognormal_particles(ng, 125.0, seed=43)
    prm = dict(omega_m0=0.3071, alpha_b0=-0.45, alpha_m0=0.05, a=0.95)
    opts = P.MgOpts(rel_tol=1e-9, max_vcycles=80, precision=prec)
    outs = []
    try:
        for side in (True, False):
            P.pm_set_step_concurrency(side)
            pos = torch.from_numpy(pos_np).cuda()
            vel = torch.zeros_like(pos)
            psi = torch.zeros((ng, ng, ng), dtype=torch.float64, device="cuda")
            chi = torch.zeros_like(psi)
            rep = P.pm_step(pos, vel, ng, prm, opts, opts, 1e-2, 1e-3, psi, chi)
            assert rep["status"] == 0
            torch.cuda.synchronize()
            outs.append((psi, chi, vel, pos))
    finally:
        P.pm_set_step_concurrency(True)
    for a, b in zip(*outs):
        assert torch.equal(a, b)
