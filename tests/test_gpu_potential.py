"""GPU parity of the NUFFT potential path (libnlf.so through the C-ABI) against the FP64 oracle.

Bar: relative max-norm error <= 1e-10 for FP64 plans and <= 1e-6 for FP32 plans, element by
element on sizes the oracle finishes in seconds; at the full 512^2 / 1024^2 sizes on sampled
outputs (type-2 at random nodes, potential at random grid points from the GPU's node values),
plus the closed forms the oracle is pinned to."""
import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import potential as op
from paper_1410_3584_amd import inputs
from gpu_util import TOL, to_dev, host_input, rel_err, oracle_u_at

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from paper_1410_3584_amd import nlf  # noqa: E402


def _case_density(n, L, seed):
    if len(n) == 2:
        rho, _ = inputs.density_2d_bumps(n, L, seed, n_bumps=4)
        return rho
    X = inputs.mesh(n, L)
    return np.exp(-(X[0] ** 2 + 2 * X[1] ** 2 + 0.5 * X[2] ** 2) / 2.0) + \
        0.3 * np.exp(-((X[0] - 1) ** 2 + (X[1] + 0.5) ** 2 + X[2] ** 2))


CASES = [
    # (n, L, kernel, prec)
    ((64, 64), (8.0, 8.0), nlf.COULOMB2D, nlf.F64),
    ((64, 64), (8.0, 8.0), nlf.LAPLACE2D, nlf.F64),
    ((64, 64), (8.0, 8.0), nlf.COULOMB2D, nlf.F32),
    ((64, 64), (8.0, 8.0), nlf.LAPLACE2D, nlf.F32),
    ((64, 32), (8.0, 6.0), nlf.COULOMB2D, nlf.F64),     # non-square grid and box
    ((32, 128), (6.0, 16.0), nlf.LAPLACE2D, nlf.F64),
    ((8, 8), (3.0, 3.0), nlf.COULOMB2D, nlf.F64),       # smallest grid: windows wrap the period
    ((128, 128), (16.0, 16.0), nlf.LAPLACE2D, nlf.F64),
    ((32, 32, 32), (8.0, 8.0, 8.0), nlf.COULOMB3D, nlf.F64),
    ((32, 32, 32), (8.0, 8.0, 8.0), nlf.COULOMB3D, nlf.F32),
    ((16, 32, 8), (4.0, 8.0, 3.0), nlf.COULOMB3D, nlf.F64),
    # 16 cells per axis: a 2 msp = 24 stencil wraps a 32-cell oversampled axis of two 16-cell
    # gather tiles (it can start and end in the same tile)
    ((16, 16), (4.0, 4.0), nlf.COULOMB2D, nlf.F64),
    ((32, 16), (6.0, 4.0), nlf.LAPLACE2D, nlf.F32),
    ((16, 16, 16), (4.0, 4.0, 4.0), nlf.COULOMB3D, nlf.F64),
]


@pytest.mark.parametrize("n,L,kernel,prec", CASES)
def test_potential_parity(n, L, kernel, prec):
    print(f"[potential parity] n={n} L={L} kernel={kernel} prec={prec}", flush=True)
    rho = _case_density(n, L, seed=7)
    plan = nlf.Plan(n, L, kernel, prec=prec)
    u = plan.potential(to_dev(rho, prec)).cpu().numpy().astype(np.float64)
    want = op.potential(host_input(rho, prec), n, L, kernel)
    assert rel_err(u, want) <= TOL[prec]


@pytest.mark.parametrize("n,L,prec,eps", [((64, 64), (8.0, 8.0), nlf.F64, 0.5),
                                          ((64, 64), (8.0, 8.0), nlf.F32, 0.5),
                                          ((128, 64), (12.0, 6.0), nlf.F64, 2.0),
                                          ((32, 32), (6.0, 6.0), nlf.F64, 0.05)])
def test_confined_potential_parity(n, L, prec, eps):
    """Confined Coulomb kernel (symbol x Jacobian erfcx(eps |k| / sqrt 2), tabulated by the plan)
    against the oracle's potential with W1 by quadrature of its defining integral."""
    print(f"[confined parity] n={n} prec={prec} eps={eps}", flush=True)
    rho = _case_density(n, L, seed=9)
    plan = nlf.Plan(n, L, nlf.CONFINED2D, prec=prec, eps=eps)
    assert plan.info.eps == eps
    u = plan.potential(to_dev(rho, prec)).cpu().numpy().astype(np.float64)
    want = op.potential(host_input(rho, prec), n, L, op.CONFINED2D, eps=eps)
    assert rel_err(u, want) <= TOL[prec]


def test_confined_gaussian_closed_form_512():
    """At 512^2 on [-16,16]^2 the GPU potential of exp(-|x|^2/sigma^2) matches the closed-form
    Hankel integral of the confined kernel at sampled points (no oracle sum involved)."""
    n, L, sigma, eps = (512, 512), (16.0, 16.0), 1.2, 0.4
    print(f"[confined closed form] n={n}", flush=True)
    X, Y = inputs.mesh(n, L)
    plan = nlf.Plan(n, L, nlf.CONFINED2D, eps=eps)
    u = plan.potential(to_dev(np.exp(-(X * X + Y * Y) / (sigma * sigma)), nlf.F64)).cpu().numpy()
    u0 = cf.confined2d_gauss_origin(sigma, eps)
    assert abs(u[256, 256] - u0) < 1e-11 * u0
    idx = [(256, 300), (100, 256), (40, 450), (0, 0), (500, 7)]
    want = cf.confined2d_gauss(np.array([np.hypot(X[i], Y[i]) for i in idx]), sigma, eps)
    assert np.max(np.abs(np.array([u[i] for i in idx]) - want)) < 1e-11 * u0


def test_confined_rejects_missing_eps():
    with pytest.raises(nlf.NlfError):
        nlf.Plan((32, 32), (6.0, 6.0), nlf.CONFINED2D)
    with pytest.raises(nlf.NlfError):
        nlf.Plan((16, 16, 16), (6.0, 6.0, 6.0), nlf.CONFINED2D, eps=0.5)


@pytest.mark.parametrize("n,L,kernel,prec", [CASES[0], CASES[2], CASES[8], CASES[10]])
def test_type2_parity(n, L, kernel, prec):
    print(f"[type2 parity] n={n} kernel={kernel} prec={prec}", flush=True)
    rho = _case_density(n, L, seed=3)
    plan = nlf.Plan(n, L, kernel, prec=prec)
    k, w = plan.nodes()
    kor, wor, _ = op.DirectPotential(n, L, kernel).k, None, None
    assert np.max(np.abs(k - kor)) < 1e-12 * np.max(np.abs(k))   # same node set, same order
    got = plan.type2(to_dev(rho, prec)).cpu().numpy()
    want = op.type2_direct(host_input(rho, prec), n, L, k)
    assert rel_err(got, want) <= TOL[prec]


@pytest.mark.parametrize("n,L,kernel,prec", [CASES[0], CASES[3], CASES[8], CASES[10]])
def test_type1_parity(n, L, kernel, prec):
    print(f"[type1 parity] n={n} kernel={kernel} prec={prec}", flush=True)
    plan = nlf.Plan(n, L, kernel, prec=prec)
    k, _ = plan.nodes()
    rng = np.random.default_rng(5)
    c = (rng.normal(size=len(k)) + 1j * rng.normal(size=len(k))) / len(k)
    cd = torch.tensor(c, dtype=plan.cdtype, device="cuda")
    got = plan.type1(cd).cpu().numpy().astype(np.float64)
    want = op.type1_direct(cd.cpu().numpy().astype(np.complex128), n, L, k)
    assert rel_err(got, want) <= TOL[prec]


@pytest.mark.parametrize("n,L,kernel,prec", [CASES[0], CASES[2], CASES[8], CASES[9]])
def test_spread_decompositions_and_autotune(n, L, kernel, prec):
    """Every spreading work decomposition (gather blocks of 64/128 candidates x work items of
    256..2048 candidates from the explicit lists, 512..2048 from the neighbour bins, and the
    LDS-atomic scatter) gives the oracle's type-1 sum; the autotuner times them all, keeps one
    of them, and the plan still agrees with the oracle.  The whole potential is checked under
    the neighbour-bin decomposition too (in 3D it switches the interpolation kernel)."""
    print(f"[spread decompositions] n={n} kernel={kernel} prec={prec}", flush=True)
    plan = nlf.Plan(n, L, kernel, prec=prec)
    assert plan.info.gather_available == 1
    k, _ = plan.nodes()
    rng = np.random.default_rng(7)
    c = (rng.normal(size=len(k)) + 1j * rng.normal(size=len(k))) / len(k)
    cd = torch.tensor(c, dtype=plan.cdtype, device="cuda")
    want = op.type1_direct(cd.cpu().numpy().astype(np.complex128), n, L, k)
    cfgs = [(nlf.SPREAD_GATHER, b, i) for b in (64, 128) for i in (256, 512, 1024, 2048)]
    assert plan.info.bins_available == 1
    cfgs += [(nlf.SPREAD_BINS, b, i) for b in (64, 128) for i in (512, 1024, 2048)]
    if prec == nlf.F32:
        # FP32 plans spread into an FP64 grid, which only the gather kernels fill
        with pytest.raises(nlf.NlfError):
            plan.set_spread(nlf.SPREAD_SCATTER)
    else:
        cfgs.append((nlf.SPREAD_SCATTER, 64, 1024))
    for mode, block, item in cfgs:
        got_cfg = plan.set_spread(mode, block, item)
        assert got_cfg[0] == mode
        got = plan.type1(cd).cpu().numpy().astype(np.float64)
        assert rel_err(got, want) <= TOL[prec], (mode, block, item)
    best, ms = plan.autotune(reps=2)
    assert ms > 0.0
    assert best in cfgs or (best[0] == nlf.SPREAD_SCATTER and any(c[0] == best[0] for c in cfgs))
    got = plan.type1(cd).cpu().numpy().astype(np.float64)
    assert rel_err(got, want) <= TOL[prec]
    with pytest.raises(nlf.NlfError):
        plan.set_spread(nlf.SPREAD_GATHER, 96, 1024)
    with pytest.raises(nlf.NlfError):
        plan.set_spread(nlf.SPREAD_GATHER, 64, 300)
    with pytest.raises(nlf.NlfError):
        plan.set_spread(nlf.SPREAD_BINS, 64, 256)     # below the allocated item minimum
    rho = _case_density(n, L, seed=11)
    want_u = op.potential(host_input(rho, prec), n, L, kernel)
    for mode in (nlf.SPREAD_BINS, nlf.SPREAD_GATHER):
        plan.set_spread(mode, 64, 1024)
        u = plan.potential(to_dev(rho, prec)).cpu().numpy().astype(np.float64)
        assert rel_err(u, want_u) <= TOL[prec], mode


@pytest.mark.parametrize("n,L,kernel,prec", [CASES[0], CASES[3], CASES[8], CASES[9], CASES[13]])
def test_deterministic_plans_repeat_bitwise(n, L, kernel, prec):
    """opts.deterministic: stored tile sums (partial sums of multi-item tiles added in a fixed
    order by a second kernel) and, in 3D, the plane-streamed interpolation: no floating-point
    atomics.  Two calls on one plan and calls
    on two plans give the same bits; the result still meets the oracle's bar; the decomposition
    cannot be changed and the autotuner only times it."""
    print(f"[deterministic] n={n} kernel={kernel} prec={prec}", flush=True)
    rho = _case_density(n, L, seed=13)
    p1 = nlf.Plan(n, L, kernel, prec=prec, deterministic=True)
    p2 = nlf.Plan(n, L, kernel, prec=prec, deterministic=True)
    assert p1.info.deterministic == 1
    r = to_dev(rho, prec)
    a = p1.potential(r).cpu().numpy()
    b = p1.potential(r).cpu().numpy()
    c = p2.potential(r).cpu().numpy()
    assert np.array_equal(a, b) and np.array_equal(a, c)
    want = op.potential(host_input(rho, prec), n, L, kernel)
    assert rel_err(a.astype(np.float64), want) <= TOL[prec]
    cfg = p1.spread_config()
    with pytest.raises(nlf.NlfError):
        p1.set_spread(nlf.SPREAD_GATHER, 64, 1024)
    got_cfg, ms = p1.autotune(reps=2)
    assert got_cfg == cfg and ms > 0.0
    assert np.array_equal(p1.potential(r).cpu().numpy(), a)


def test_deterministic_split_and_ground_state_repeat_bitwise():
    """A deterministic split plan (its ball plan inherits the option) and ground states on a
    deterministic plan (including the FP64 twin of the mixed schedule) repeat bit for bit."""
    print("[deterministic split + ground state]", flush=True)
    n, L = (64, 64, 64), (8.0, 8.0, 8.0)
    X = inputs.mesh(n, L)
    r = torch.tensor(np.exp(-(X[0] ** 2 + X[1] ** 2 + X[2] ** 2)), dtype=torch.float64, device="cuda")
    sp = nlf.Plan(n, L, nlf.COULOMB3D, split=True, deterministic=True)
    a = sp.potential(r).cpu().numpy()
    assert np.array_equal(a, sp.potential(r).cpu().numpy())
    ref = nlf.Plan(n, L, nlf.COULOMB3D, split=True).potential(r).cpu().numpy()
    assert rel_err(a, ref) <= 1e-12
    g = nlf.Plan((64, 64), (16.0, 16.0), nlf.COULOMB2D, prec=nlf.F32, batch=2, deterministic=True)
    runs = [g.ground_state([40.0, 300.0], [(1.0, 1.3), (1.0, 0.9)], tau=0.25, eps0=1e-10, mixed=True)
            for _ in range(2)]
    assert runs[0][2] == nlf.OK and runs[1][2] == nlf.OK
    assert np.array_equal(runs[0][0].cpu().numpy(), runs[1][0].cpu().numpy())
    assert [s["E"] for s in runs[0][1]] == [s["E"] for s in runs[1][1]]
    assert [s["iters"] for s in runs[0][1]] == [s["iters"] for s in runs[1][1]]


def test_deterministic_neighbour_bins_256():
    """A deterministic plain-ball plan at 256^3, where the spreading reads neighbour-bin streams:
    two calls give the same bits, and the result equals the default plan's to rounding."""
    print("[deterministic neighbour bins 256^3]", flush=True)
    n, L = (256, 256, 256), (12.0, 12.0, 12.0)
    rho = np.abs(inputs.psi0_phase_modulated(n, L, seed=0)) ** 2
    rd = to_dev(rho, 0)
    pd = nlf.Plan(n, L, nlf.COULOMB3D, deterministic=True)
    assert pd.spread_config()[0] == nlf.SPREAD_BINS
    a = pd.potential(rd)
    b = pd.potential(rd)
    assert torch.equal(a, b)
    del pd
    ref = nlf.Plan(n, L, nlf.COULOMB3D).potential(rd)
    assert float((a - ref).abs().max() / ref.abs().max()) <= 1e-12


def test_neighbour_bins_match_explicit_lists_512():
    """At 512^2 (both decompositions available) the neighbour-bin gather and the explicit
    candidate lists give the same potential up to FP64 rounding (the extra candidates of the
    bins add only weights below the stencil's truncation level)."""
    n, L = (512, 512), (16.0, 16.0)
    print(f"[bins vs lists] n={n}", flush=True)
    rho = _case_density(n, L, seed=5)
    plan = nlf.Plan(n, L, nlf.COULOMB2D)
    assert plan.info.gather_available == 1 and plan.info.bins_available == 1
    out = {}
    for mode in (nlf.SPREAD_GATHER, nlf.SPREAD_BINS):
        plan.set_spread(mode, 64, 1024)
        out[mode] = plan.potential(to_dev(rho, nlf.F64)).cpu().numpy()
    assert rel_err(out[nlf.SPREAD_BINS], out[nlf.SPREAD_GATHER]) <= 1e-12


def test_batch_matches_single():
    n, L = (64, 64), (8.0, 8.0)
    rhos = np.stack([_case_density(n, L, s) for s in (1, 2, 3)])
    for kernel in (nlf.COULOMB2D, nlf.LAPLACE2D):
        pb = nlf.Plan(n, L, kernel, batch=3)
        ub = pb.potential(to_dev(rhos, 0)).cpu().numpy()
        for i in range(3):
            want = op.potential(rhos[i], n, L, kernel)
            assert rel_err(ub[i], want) <= 1e-10


def test_zero_density_gives_zero():
    for n, L, kernel in [((32, 32), (8.0, 8.0), nlf.LAPLACE2D), ((16, 16, 16), (4.0,) * 3, nlf.COULOMB3D)]:
        plan = nlf.Plan(n, L, kernel)
        u = plan.potential(torch.zeros(n, dtype=torch.float64, device="cuda"))
        assert float(u.abs().max()) == 0.0


def test_single_point_density():
    """A density that is one grid value: the most concentrated input the grid can hold."""
    n, L = (32, 32), (8.0, 8.0)
    rho = np.zeros(n)
    rho[20, 9] = 1.0
    for kernel in (nlf.COULOMB2D, nlf.LAPLACE2D):
        u = nlf.Plan(n, L, kernel).potential(to_dev(rho, 0)).cpu().numpy()
        assert rel_err(u, op.potential(rho, n, L, kernel)) <= 1e-10


def test_repeat_calls_identical_structure():
    """Two calls on the same plan agree to rounding (the spread grid is cleared between calls: a
    stale grid would double the second result).  The FP64 atomics of the spreading add in no fixed
    order, so the two calls may differ by some tens of ulps (1.06e-14 seen)."""
    n, L = (64, 64), (8.0, 8.0)
    rho = to_dev(_case_density(n, L, 9), 0)
    plan = nlf.Plan(n, L, nlf.COULOMB2D)
    a = plan.potential(rho).cpu().numpy()
    b = plan.potential(rho).cpu().numpy()
    assert rel_err(a, b) <= 1e-13


def test_invalid_arguments_rejected():
    with pytest.raises(nlf.NlfError) as e:
        nlf.Plan((48, 48), (8.0, 8.0), nlf.COULOMB2D)
    assert e.value.status == nlf.EUNSUPPORTED
    with pytest.raises(nlf.NlfError) as e:
        nlf.Plan((32, 32, 32), (8.0,) * 3, nlf.COULOMB2D)
    assert e.value.status == nlf.EUNSUPPORTED
    with pytest.raises(nlf.NlfError) as e:
        nlf.Plan((32, 32), (8.0, 8.0), nlf.COULOMB2D, P=100.0)
    assert e.value.status == nlf.EINVAL
    plan = nlf.Plan((32, 32), (8.0, 8.0), nlf.COULOMB2D)
    with pytest.raises(ValueError):
        plan.potential(torch.zeros((32, 32), dtype=torch.float32, device="cuda"))


# ---- full-size 2D workload (512^2 on [-16,16]^2), sampled ------------------------------------

@pytest.mark.parametrize("kernel,prec", [(nlf.COULOMB2D, nlf.F64), (nlf.LAPLACE2D, nlf.F64),
                                         (nlf.COULOMB2D, nlf.F32), (nlf.LAPLACE2D, nlf.F32)])
def test_full_size_2d_sampled(kernel, prec):
    print(f"[full 512^2 sampled] kernel={kernel} prec={prec}", flush=True)
    n, L, rho, _ = inputs.potential_2d_512(seed=1)
    plan = nlf.Plan(n, L, kernel, prec=prec)
    rd = to_dev(rho, prec)
    rhost = host_input(rho, prec)
    k, w = plan.nodes()
    rng = np.random.default_rng(11)
    # (1) type-2 at 384 random nodes (full sum over the grid for each)
    rh = plan.type2(rd).cpu().numpy().astype(np.complex128)
    sel = rng.choice(len(k), 384, replace=False)
    want = op.type2_direct(rhost, n, L, k[sel])
    assert np.max(np.abs(rh[sel] - want)) <= TOL[prec] * np.max(np.abs(rh))
    # (2) potential at 96 random grid points from the GPU's rhohat through the oracle's symbol
    dp = op.DirectPotential.__new__(op.DirectPotential)
    kmag = np.linalg.norm(k, axis=1)
    m0 = m1 = None
    sigma = plan.info.sigma
    if kernel == nlf.LAPLACE2D:
        m0, m1 = op.moments(rhost, n, L)
    c = op.symbol_coeffs(kernel, k, w, kmag, rh, m0, m1, sigma)
    pts = [tuple(rng.integers(0, n[i]) for i in range(2)) for _ in range(96)] + [(256, 256), (0, 0), (511, 3)]
    u = plan.potential(rd).cpu().numpy().astype(np.float64)
    want_u = oracle_u_at(pts, c, k, n, L, kernel, rho=rhost, sigma=sigma)
    got_u = np.array([u[p] for p in pts])
    assert np.max(np.abs(got_u - want_u)) <= TOL[prec] * np.max(np.abs(u))


def test_full_size_2d_closed_form():
    """The 2D workload's density is a sum of Gaussians, so both kernels have closed forms
    (Examples 2.2/2.3 plus superposition); FP64 at 512^2 meets them to ~1e-12."""
    n, L, rho, bumps = inputs.potential_2d_512(seed=1)
    xs = inputs.axes(n, L)
    pts = [(256, 256), (300, 200), (100, 400), (10, 500), (256, 300)]
    for kernel in (nlf.COULOMB2D, nlf.LAPLACE2D):
        u = nlf.Plan(n, L, kernel).potential(to_dev(rho, 0)).cpu().numpy()
        for p in pts:
            x, y = xs[0][p[0]], xs[1][p[1]]
            if kernel == nlf.COULOMB2D:
                v = float(cf.coulomb2d_gauss_aniso(x, y, 1.0, 2.0))
                v += sum(a * float(cf.coulomb2d_gauss(np.hypot(x - c[0], y - c[1]), wb)) for a, c, wb in bumps)
            else:
                v = float(cf.laplace2d_gauss_aniso(x, y, 1.0, 0.5))
                v += sum(a * float(cf.laplace2d_gauss(np.hypot(x - c[0], y - c[1]), wb)) for a, c, wb in bumps)
            assert abs(u[p] - v) <= 1e-9 * np.max(np.abs(u)), (kernel, p, u[p], v)


def test_largest_grid_1024_sampled():
    """n = 1024 per axis (2048-point FFT lines on the oversampled grid), FP64 Coulomb."""
    n, L = (1024, 1024), (16.0, 16.0)
    rho, _ = inputs.density_2d_bumps(n, L, seed=4, n_bumps=3)
    plan = nlf.Plan(n, L, nlf.COULOMB2D, n_r=256, n_phi=512)
    k, w = plan.nodes()
    rd = to_dev(rho, 0)
    rh = plan.type2(rd).cpu().numpy()
    rng = np.random.default_rng(2)
    sel = rng.choice(len(k), 128, replace=False)
    assert np.max(np.abs(rh[sel] - op.type2_direct(rho, n, L, k[sel]))) <= 1e-10 * np.max(np.abs(rh))
    c = op.symbol_coeffs(nlf.COULOMB2D, k, w, np.linalg.norm(k, axis=1), rh)
    u = plan.potential(rd).cpu().numpy()
    pts = [tuple(rng.integers(0, 1024, size=2)) for _ in range(32)] + [(512, 512), (0, 1023)]
    want = oracle_u_at(pts, c, k, n, L, nlf.COULOMB2D)
    assert np.max(np.abs(np.array([u[p] for p in pts]) - want)) <= 1e-10 * np.max(np.abs(u))


def test_dynamics_workload_256_sampled():
    """3D dynamics workload at full size: 256^3 on [-12,12]^3, Coulomb kernel, 256x256x512 nodes,
    rho = |psi0|^2 of the seeded phase-modulated Gaussian.  Type-2 at sampled nodes and the
    potential at sampled grid points (from the GPU's node values over the full node set) against
    the oracle's direct sums, <= 1e-10."""
    print("[256^3 sampled]", flush=True)
    n, L = (256, 256, 256), (12.0, 12.0, 12.0)
    psi0 = inputs.psi0_phase_modulated(n, L, seed=0)
    rho = np.abs(psi0) ** 2
    plan = nlf.Plan(n, L, nlf.COULOMB3D)
    k, w = plan.nodes()
    rd = to_dev(rho, 0)
    rh = plan.type2(rd).cpu().numpy()
    rng = np.random.default_rng(3)
    sel = rng.choice(len(k), 16, replace=False)
    scale = np.max(np.abs(rh))
    assert np.max(np.abs(rh[sel] - op.type2_direct(rho, n, L, k[sel]))) <= 1e-10 * scale
    c = op.symbol_coeffs(nlf.COULOMB3D, k, w, np.linalg.norm(k, axis=1), rh)
    del rh
    u = plan.potential(rd).cpu().numpy()
    pts = [tuple(rng.integers(0, 256, size=3)) for _ in range(6)] + [(128, 128, 128), (0, 255, 7)]
    want = oracle_u_at(pts, c, k, n, L, nlf.COULOMB3D)
    assert np.max(np.abs(np.array([u[p] for p in pts]) - want)) <= 1e-10 * np.max(np.abs(u))


def test_coulomb3d_workload_closed_form():
    """3D check workload: rho = e^{-|x|^2} on 32^3 of [-8,8]^3, 32x32x64 nodes; continuum error
    is the ball/angular floor (< 5e-5, see the oracle pins), parity <= 1e-10."""
    n, L, rho = inputs.coulomb3d_gauss_32()
    u = nlf.Plan(n, L, nlf.COULOMB3D).potential(to_dev(rho, 0)).cpu().numpy()
    X = inputs.mesh(n, L)
    R = np.sqrt(sum(x * x for x in X))
    assert rel_err(u, cf.coulomb3d_gauss(R, 1.0)) < 5e-5
