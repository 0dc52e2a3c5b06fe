"""GPU parity of the other schemes of Sec. 2.2 (hydro_advance_ext) against
the oracle: MHM and CTU; PLM and PPM on primitive or characteristic
variables; generalized minmod, van Leer, van Albada and hybrid limiters;
HLLC, Roe and HLLE.  Bars as for the default step: |g - o| <= tol (|o| +
ref_f) per cell (momentum on one scale) and, in FP64, rho and E within tol
relative per cell; tol = 1e-12 (FP64) and 1e-5 (FP32, oracle started from
the FP32-rounded state); unphysical counts equal.  Also: the default word
on this path agrees with the fused kernels; chunked workspaces give the
same bits as one chunk; the 256^3 shear layer at sampled groups."""

import sys

import numpy as np
import pytest

import oracle
from paper_1712_07070_amd import workloads as W
from tests.oracle_runs import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {np.float64: 1e-12, np.float32: 1e-5}
MHM, CTU = oracle.SCHEME_MHM, oracle.SCHEME_CTU
SCHEMES = {
    "mhm-plm-gminmod-hllc": MHM,
    "vanleer": MHM | oracle.LIMITER_VANLEER,
    "vanalbada": MHM | oracle.LIMITER_VANALBADA,
    "hybrid": MHM | oracle.LIMITER_HYBRID,
    "char": MHM | oracle.CHARACTERISTIC,
    "char-vanleer": MHM | oracle.CHARACTERISTIC | oracle.LIMITER_VANLEER,
    "ppm": MHM | oracle.PPM,
    "ppm-char-hybrid": MHM | oracle.PPM | oracle.CHARACTERISTIC | oracle.LIMITER_HYBRID,
    "roe": MHM | oracle.RIEMANN_ROE,
    "hlle": MHM | oracle.RIEMANN_HLLE,
    "hlle-davis": MHM | oracle.RIEMANN_HLLE | oracle.WAVESPEED_DAVIS,
    "first-order-roe": MHM | oracle.FIRST_ORDER | oracle.RIEMANN_ROE,
    "ctu": CTU,
    "ctu-roe": CTU | oracle.RIEMANN_ROE,
    "ctu-ppm-char-hybrid": CTU | oracle.PPM | oracle.CHARACTERISTIC | oracle.LIMITER_HYBRID,
    "ctu-hlle-vanalbada": CTU | oracle.RIEMANN_HLLE | oracle.LIMITER_VANALBADA,
}


@pytest.fixture(scope="module")
def hydro():
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    from paper_1712_07070_amd import hydro as h
    h.load()
    return h


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else a.astype(dtype))
    return torch.from_numpy(a).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def cfl_dt(U, ng, bc, dx, gamma):
    return float(oracle.dt_patch(oracle.fill_ghosts(U, ng, 3, bc), dx, gamma, 0.5).min())


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("name", list(SCHEMES))
def test_ext_step_matches_oracle(hydro, name, dtype):
    say("ext step", name, dtype.__name__)
    sch = SCHEMES[name]
    lv = W.white_noise(32)
    U = lv.U.astype(dtype).astype(np.float64)
    pad = oracle.fill_ghosts(U, lv.ng, 3, lv.bc)
    dt = cfl_dt(U, lv.ng, lv.bc, lv.dx, lv.gamma)
    ref, nb_ref = oracle.step_any(pad, dt, lv.dx, lv.gamma, 1.5, sch)
    n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = hydro.advance_ext(dev(pad, dtype), dt, lv.dx, lv.gamma, sch, n_bad=n_bad)
    assert_parity(host(got), ref, TOL[dtype], name)
    assert int(host(n_bad)[0]) == nb_ref == 0


@pytest.mark.parametrize("name", ["ppm-char-hybrid", "ctu-roe", "roe", "hlle"])
@pytest.mark.parametrize("theta", [1.0, 2.0])
def test_ext_theta_and_sod(hydro, name, theta):
    """Sod tube (outflow ends, strong discontinuities: limiter and solver
    branches everywhere) at theta 1 and 2."""
    say("ext sod", name, theta)
    sch = SCHEMES[name]
    lv = W.sod_tube(64)
    pad = oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc)
    dt = cfl_dt(lv.U, lv.ng, lv.bc, lv.dx, lv.gamma)
    ref, nb = oracle.step_any(pad, dt, lv.dx, lv.gamma, theta, sch)
    got = hydro.advance_ext(dev(pad), dt, lv.dx, lv.gamma, sch, theta=theta)
    assert_parity(host(got), ref, 1e-12, name)
    assert nb == 0


def test_ext_unphysical_counts(hydro):
    """Low-pressure white noise: the counts of faces with unphysical input
    states and of unphysical updated cells equal the oracle's."""
    say("ext unphysical counts")
    rng = np.random.default_rng(0)
    n = 32
    rho = rng.uniform(0.05, 2, (n, n, n))
    p = np.exp(rng.uniform(np.log(1e-3), np.log(2.0), (n, n, n)))
    v = rng.normal(0, 0.5, (3, n, n, n))
    U = W.grid_to_groups(W.conserved(rho, v[0], v[1], v[2], p, 5.0 / 3.0))
    ng, bc, dx = (2, 2, 2), (0,) * 6, 1.0 / n
    pad = oracle.fill_ghosts(U, ng, 3, bc)
    dt = cfl_dt(U, ng, bc, dx, 5.0 / 3.0)
    for name in ("roe", "ctu", "ppm"):
        ref, nb = oracle.step_any(pad, dt, dx, 5.0 / 3.0, 1.5, SCHEMES[name])
        n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
        hydro.advance_ext(dev(pad), dt, dx, 5.0 / 3.0, SCHEMES[name], n_bad=n_bad)
        assert int(host(n_bad)[0]) == nb > 0, name


def test_ext_default_word_agrees_with_fused_step(hydro):
    lv = W.white_noise(32)
    pad = dev(oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc))
    dt = cfl_dt(lv.U, lv.ng, lv.bc, lv.dx, lv.gamma)
    a = host(hydro.advance(pad, dt, lv.dx, lv.gamma))
    b = host(hydro.advance_ext(pad, dt, lv.dx, lv.gamma, MHM))
    assert_parity(b, a, 1e-12, "ext vs fused")


@pytest.mark.parametrize("name", ["ctu-ppm-char-hybrid", "ppm", "roe"])
def test_ext_chunked_workspace_and_determinism(hydro, name):
    """A workspace for 3 groups (the 8 groups run in chunks of 3, 3, 2) gives
    the same bits as one for all 8, and repeated runs the same bits (a word
    of the fused kernel, roe, needs no workspace and ignores it)."""
    sch = SCHEMES[name]
    lv = W.white_noise(32)
    pad = dev(oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc))
    dt = cfl_dt(lv.U, lv.ng, lv.bc, lv.dx, lv.gamma)
    full = host(hydro.advance_ext(pad, dt, lv.dx, lv.gamma, sch))
    again = host(hydro.advance_ext(pad, dt, lv.dx, lv.gamma, sch))
    work = hydro.ext_workspace(3, 3, torch.float64, sch)
    part = host(hydro.advance_ext(pad, dt, lv.dx, lv.gamma, sch, work=work))
    assert np.array_equal(full, again) and np.array_equal(full, part)


def test_ext_argument_errors(hydro):
    lv = W.white_noise(16)
    pad3 = dev(oracle.fill_ghosts(lv.U, lv.ng, 3, lv.bc))
    pad2 = dev(oracle.fill_ghosts(lv.U, lv.ng, 2, lv.bc))
    with pytest.raises(hydro.HydroError):   # PPM needs 3 ghost layers
        hydro.advance_ext(pad2, 1e-3, lv.dx, lv.gamma, MHM | oracle.PPM,
                          work=torch.empty(1 << 24, dtype=torch.uint8, device="cuda"))
    with pytest.raises(hydro.HydroError):   # solver id 3 does not exist
        hydro.advance_ext(pad3, 1e-3, lv.dx, lv.gamma, MHM | (3 << 16),
                          work=torch.empty(1 << 24, dtype=torch.uint8, device="cuda"))
    with pytest.raises(hydro.HydroError):   # workspace below one group
        hydro.advance_ext(pad3, 1e-3, lv.dx, lv.gamma, CTU, work=torch.empty(1024, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("name", ["ppm-char-hybrid", "ctu-roe", "char-vanleer", "hlle-davis"])
def test_ext_shear_layer_256_sampled(hydro, name, dtype):
    """The 256^3 shear layer (4096 groups) in one call; 12 sampled groups
    against the oracle on their own padded blocks (PPM and CTU words through
    the chain of kernels, the others through the fused kernel)."""
    say("ext 256^3", name, dtype.__name__)
    sch = SCHEMES[name]
    lv = W.shear_layer(256)
    U = dev(lv.U, dtype)
    pad = hydro.fill_ghosts(U, lv.ng, 3, lv.bc)
    del U
    dt = float(hydro.cfl_dt(pad, lv.dx, lv.gamma, 0.5).min())
    got = hydro.advance_ext(pad, dt, lv.dx, lv.gamma, sch)
    rng = np.random.default_rng(5)
    gs = np.sort(rng.choice(lv.n_groups, 12, replace=False))
    p = host(pad[torch.from_numpy(gs).cuda()]).astype(np.float64)
    ref, nb = oracle.step_any(p, dt, lv.dx, lv.gamma, 1.5, sch)
    assert_parity(host(got[torch.from_numpy(gs).cuda()]), ref, TOL[dtype], name)
    assert nb == 0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("name", ["mhm-plm-gminmod-hllc", "ppm-char-hybrid", "ctu-roe"])
@pytest.mark.parametrize("xi", [0.01, 1e300])
def test_ext_dual_energy_matches_oracle(hydro, name, dtype, xi):
    """Dual energy (6 fields, field 5 the entropy s = p / rho^(gamma-1)):
    xi = 0.01 (the paper's typical threshold) and xi = inf (E always from s);
    the entropy field within tol of its largest value."""
    from tests.test_oracle_dual_energy import with_entropy
    say("ext dual energy", name, dtype.__name__, xi)
    sch = SCHEMES[name] | oracle.DUAL_ENERGY
    lv = W.white_noise(32)
    U6 = with_entropy(lv.U).astype(dtype).astype(np.float64)
    pad5 = oracle.fill_ghosts(U6[:, :5], lv.ng, 3, lv.bc)
    pads = oracle.fill_ghosts(np.repeat(U6[:, 5:], 5, axis=1), lv.ng, 3, lv.bc)[:, :1]
    pad = np.concatenate([pad5, pads], axis=1)
    dt = cfl_dt(U6[:, :5], lv.ng, lv.bc, lv.dx, lv.gamma)
    ref, nb = oracle.step_any_de(pad, dt, lv.dx, lv.gamma, 1.5, sch, xi)
    n_bad = torch.zeros(1, dtype=torch.int32, device="cuda")
    got = host(hydro.advance_ext(dev(pad, dtype), dt, lv.dx, lv.gamma, sch, n_bad=n_bad, xi=xi)).astype(np.float64)
    assert_parity(got[:, :5], ref[:, :5], TOL[dtype], name)
    assert np.abs(got[:, 5] - ref[:, 5]).max() <= TOL[dtype] * np.abs(ref[:, 5]).max(), name
    assert int(host(n_bad)[0]) == nb == 0


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("name", ["default", "davis", "first-order"])
def test_fused_face_fluxes_match_oracle(hydro, name, dtype):
    """Words the fused kernel computes (MHM, primitive PLM, generalized
    minmod, HLLC) run there, with no workspace; the patch-boundary face
    fluxes it reports equal the oracle's within tol (|o| + max |o| of the
    field), the state as for the other words."""
    sch = {"default": MHM, "davis": MHM | oracle.WAVESPEED_DAVIS, "first-order": MHM | oracle.FIRST_ORDER}[name]
    say("fused face fluxes", name, dtype.__name__)
    assert hydro.load().hydro_ext_workspace_bytes(8, 3, 0, sch) == 0
    lv = W.white_noise(32)
    U = lv.U.astype(dtype).astype(np.float64)
    pad = oracle.fill_ghosts(U, lv.ng, 3, lv.bc)
    dt = cfl_dt(U, lv.ng, lv.bc, lv.dx, lv.gamma)
    ref, ffo, nb = oracle.step_any_flux(pad, dt, lv.dx, lv.gamma, 1.5, sch)
    ff = torch.full((lv.n_groups, 9, 5, 16, 16), float("nan"), dtype=torch.float64 if dtype == np.float64 else
                    torch.float32, device="cuda")
    got = hydro.advance_ext(dev(pad, dtype), dt, lv.dx, lv.gamma, sch, face_flux=ff)
    assert_parity(host(got), ref, TOL[dtype], name)
    f = host(ff).astype(np.float64)
    assert np.isfinite(f).all()
    scale = np.abs(ffo).max(axis=(0, 1, 3, 4))[None, None, :, None, None]
    err = np.abs(f - ffo) / (np.abs(ffo) + scale)
    assert err.max() <= TOL[dtype], (name, float(err.max()))
    assert nb == 0
