"""GPU parity of the IRN-PICCS solve and its pieces against the FP64 oracle.

The same seeded inputs go to both sides; the GPU runs float32 storage with
float64 Krylov scalars, the oracle float64 throughout.  Tolerances: weights
1e-5 (float32 sqrt chain); solves 1e-4 relative L2 after the full iteration
count (float32 rounding amplified by the Krylov recurrence, measured against
the float64 iterates).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

SOLVE_TOL = 1e-4


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_08574_amd import cbct
    return cbct


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def c1_inputs(orc):
    from paper_2509_08574_amd import synth
    d = synth.geometry("c1")
    og = orc.Geometry.from_dict(d)
    prior, cur = synth.c1_case()
    sp = synth.SOLVE_PARAMS["c1"]
    b = synth.noisy_line_integrals(orc.forward(og, cur), sp["I0"], seed=101)
    # both sides see the same float32-rounded inputs
    b = b.astype(np.float32).astype(np.float64)
    prior = prior.astype(np.float32).astype(np.float64)
    return d, og, prior, cur, b, sp


def test_weights_parity(orc, lib):
    d, og, prior, cur, b, sp = c1_inputs(orc)
    gg = lib.Geometry.from_dict(d)
    x = cur.astype(np.float32).astype(np.float64)
    w1o, w2o = orc.weights(x, prior, sp["tau"])
    w1, w2 = lib.weights(gg, dev(x), dev(prior), sp["tau"])
    assert rel(host(w1), w1o) <= 1e-5
    assert rel(host(w2), w2o) <= 1e-5


@pytest.mark.parametrize("ny", [1, 2, 7, 8])
def test_weights_parity_plane_pairs(orc, lib, ny):
    """The weights kernel takes two y-planes per thread: odd and even plane counts
    (a lone last plane, a single plane), ragged x and z, against the oracle."""
    rng = np.random.default_rng(30 + ny)
    d = dict(nx=13, ny=ny, nz=70, vx=1.0, vy=1.0, vz=1.0, nu=8, nv=8, du=1.0, dv=1.0,
             dso=60.0, dsd=100.0, n_views=2)
    gg = lib.Geometry.from_dict(d)
    x = rng.uniform(size=gg.vol_shape).astype(np.float32).astype(np.float64)
    xp = (x + 0.2 * rng.uniform(size=gg.vol_shape)).astype(np.float32).astype(np.float64)
    w1o, w2o = orc.weights(x, xp, 0.1)
    w1, w2 = lib.weights(gg, dev(x), dev(xp), 0.1)
    assert rel(host(w1), w1o) <= 1e-5
    assert rel(host(w2), w2o) <= 1e-5


def _gpu_solve(lib, d, b, xp, x0, p):
    gg = lib.Geometry.from_dict(d)
    x = dev(x0)
    x, rep = lib.solve(gg, dev(b), dev(xp), x, p)
    return host(x), rep


def test_c1_irn_piccs_parity(orc, lib):
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"],
                        sp["n_inner"])
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"])
    xg, rep = _gpu_solve(lib, d, b, prior, prior, p)
    assert rep["inner_done"] == len(ref.phibar) == sp["n_outer"] * sp["n_inner"]
    assert rep["outer_done"] == sp["n_outer"]
    assert rep["breakdown"] == 0
    assert rel(xg, ref.x) <= SOLVE_TOL
    np.testing.assert_allclose(rep["phibar"], ref.phibar, rtol=SOLVE_TOL)
    # the reconstruction moved towards the current object
    assert np.linalg.norm(xg - cur) < np.linalg.norm(prior - cur)


def test_plain_lsqr_special_case(orc, lib):
    """alpha = lambda = 0: one outer step is plain LSQR on A x = b."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, 0.0, 0.0, sp["tau"], 1, 8)
    xg, rep = _gpu_solve(lib, d, b, prior, prior, lib.SolveParams(0.0, 0.0, sp["tau"], 1, 8))
    assert rel(xg, ref.x) <= SOLVE_TOL
    np.testing.assert_allclose(rep["phibar"], ref.phibar, rtol=SOLVE_TOL)


def test_irn_tv_special_case(orc, lib):
    """lambda = 0: IRN-TV."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], 0.0, sp["tau"], 2, 4)
    xg, _ = _gpu_solve(lib, d, b, prior, prior,
                       lib.SolveParams(sp["alpha"], 0.0, sp["tau"], 2, 4))
    assert rel(xg, ref.x) <= SOLVE_TOL


def test_prior_fixed_point(orc, lib):
    """b = A x_p, x_0 = x_p, alpha = 0: the prior is (numerically) a fixed point."""
    from paper_2509_08574_amd import synth
    d = synth.geometry("c1")
    og = orc.Geometry.from_dict(d)
    prior, _ = synth.c1_case()
    prior = prior.astype(np.float32).astype(np.float64)
    b = orc.forward(og, prior)
    xg, rep = _gpu_solve(lib, d, b, prior, prior, lib.SolveParams(0.0, 1.0, 0.1, 2, 4))
    assert rel(xg, prior) <= 1e-5


def test_non_finite_input_returns_numeric_error(orc, lib):
    """NaN in b, or Inf in x_0: the solve stops at the first non-finite norm and
    returns CBCT_ERR_NUMERIC (with a report); x keeps its last finite iterate."""
    import torch
    d, og, prior, cur, b, sp = c1_inputs(orc)
    gg = lib.Geometry.from_dict(d)
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], 1, 3)
    bad = b.copy()
    bad.reshape(-1)[777] = np.nan
    x = dev(prior)
    with pytest.raises(lib.CbctError) as ei:
        lib.solve(gg, dev(bad), dev(prior), x, p)
    assert ei.value.code == lib.ERR_NUMERIC
    assert torch.isfinite(x).all()
    assert np.array_equal(host(x), prior)   # stopped before the first update
    x0 = prior.copy()
    x0.reshape(-1)[4321] = np.inf
    x = dev(x0)
    with pytest.raises(lib.CbctError) as ei:
        lib.solve(gg, dev(b), dev(prior), x, p)
    assert ei.value.code == lib.ERR_NUMERIC
    # the same call without a report only enqueues; a finite solve after it is clean
    x = dev(prior)
    lib.solve(gg, dev(bad), dev(prior), x, p, report=False)
    x = dev(prior)
    _, rep = lib.solve(gg, dev(b), dev(prior), x, p)
    assert rep["inner_done"] == 3 and rep["breakdown"] == 0


def test_solve_is_deterministic(orc, lib):
    d, og, prior, cur, b, sp = c1_inputs(orc)
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], 2, 3)
    x1, r1 = _gpu_solve(lib, d, b, prior, prior, p)
    x2, r2 = _gpu_solve(lib, d, b, prior, prior, p)
    assert np.array_equal(x1, x2)
    assert r1["phibar"] == r2["phibar"]


def test_odd_geometry_solve(orc, lib):
    """Ragged sizes: several 64-row blocks, odd volume, non-uniform angles."""
    rng = np.random.default_rng(9)
    d = dict(nx=13, ny=11, nz=17, vx=1.0, vy=1.0, vz=1.0, nu=23, nv=70, du=1.3, dv=0.5,
             dso=60.0, dsd=100.0, n_views=11,
             angles=list(np.sort(rng.uniform(0, 2 * np.pi, 11))))
    og = orc.Geometry.from_dict(d)
    xp = rng.uniform(size=og.vol_shape).astype(np.float32).astype(np.float64)
    xt = xp + 0.3 * (rng.uniform(size=og.vol_shape) > 0.95)
    b = orc.forward(og, xt).astype(np.float32).astype(np.float64)
    ref = orc.irn_piccs(og, b, xp, xp, 0.5, 1.5, 0.2, 2, 4)
    xg, rep = _gpu_solve(lib, d, b, xp, xp, lib.SolveParams(0.5, 1.5, 0.2, 2, 4))
    assert rel(xg, ref.x) <= SOLVE_TOL


@pytest.mark.parametrize("nv, dv", [(300, 0.7), (384, 0.55), (512, 0.5)])
def test_solve_with_several_rows_per_lane(orc, lib, nv, dv):
    """Detector heights at which the forward projector takes two, three and four
    rows per lane (its solver form fuses the u update and the |u|^2 partials);
    a tall volume puts data on every row.  FP32 and mixed BF16."""
    rng = np.random.default_rng(nv)
    d = dict(nx=10, ny=10, nz=100, vx=1.0, vy=1.0, vz=1.0, nu=12, nv=nv, du=2.0, dv=dv,
             dso=100.0, dsd=200.0, n_views=12)
    og = orc.Geometry.from_dict(d)
    xp = rng.uniform(size=og.vol_shape).astype(np.float32).astype(np.float64)
    xt = xp + 0.3 * (rng.uniform(size=og.vol_shape) > 0.9)
    b = orc.forward(og, xt).astype(np.float32).astype(np.float64)
    ref = orc.irn_piccs(og, b, xp, xp, 0.5, 1.5, 0.2, 2, 4)
    xg, rep = _gpu_solve(lib, d, b, xp, xp, lib.SolveParams(0.5, 1.5, 0.2, 2, 4))
    assert rep["inner_done"] == 8
    assert rel(xg, ref.x) <= SOLVE_TOL
    xm, _ = _gpu_solve(lib, d, b, xp, xp,
                       lib.SolveParams(0.5, 1.5, 0.2, 2, 4, precision=lib.PREC_MIXED_BF16))
    assert rel(xm, ref.x) <= 1e-3


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_mixed_precision_solve_within_1e3_of_fp64(orc, lib, prec):
    """16-bit projector operand, fp32 accumulation, fp64 Krylov scalars: <= 1e-3 vs FP64."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"],
                        sp["n_inner"])
    pr = lib.PREC_MIXED_BF16 if prec == "bf16" else lib.PREC_MIXED_F16
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                        precision=pr)
    xg, rep = _gpu_solve(lib, d, b, prior, prior, p)
    err = rel(xg, ref.x)
    print(f"{prec}: rel L2 vs FP64 oracle {err:.2e}")
    assert err <= 1e-3
    assert rep["inner_done"] == sp["n_outer"] * sp["n_inner"]


# A small volume seen on a tall detector (1024 rows of 0.25 mm), the shape on
# which the adjoint's 16-bit input pays most: a 16 x 16 column tile's per-view
# detector footprint in float32, (16 h sqrt(2) DSD / (DSO du) + 2) x nv x 4 B, is
# 36 x 1024 x 4 B = 147 KB (at 256^3 it is 91 KB, at 512x512x400 193 KB).
TALL = dict(nx=20, ny=20, nz=40, vx=1.0, vy=1.0, vz=0.5, nu=24, nv=1024, du=1.0, dv=0.25,
            dso=400.0, dsd=600.0, n_views=9)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "f16"])
def test_mixed_adjoint_16bit_input_against_oracle(orc, lib, prec):
    """The adjoint's 16-bit u-hat (bf16, scaled fp16) through a whole IRN-PICCS
    solve, against the FP64 oracle: 1e-3 for the mixed forms, 1e-4 for FP32."""
    from paper_2509_08574_amd import synth
    og = orc.Geometry.from_dict(TALL)
    prior, _ = synth.ellipsoid_phantom(og.vol_shape, 6, (2.0, 8.0), seed=21)
    cur = prior.copy()
    synth.add_cylinder(cur, (10.0, 10.0, 20.0), (0.2, 0.3, 0.9), 1.0, 20.0, 2.0)
    b = synth.noisy_line_integrals(orc.forward(og, cur), 1e5, seed=22)
    b = b.astype(np.float32).astype(np.float64)
    prior = prior.astype(np.float32).astype(np.float64)
    ref = orc.irn_piccs(og, b, prior, prior, 1.0, 1.0, 0.1, 2, 3)
    pr = {"fp32": lib.PREC_FP32, "bf16": lib.PREC_MIXED_BF16_ADJ16,
          "f16": lib.PREC_MIXED_F16_ADJ16}[prec]
    xg, rep = _gpu_solve(lib, TALL, b, prior, prior, lib.SolveParams(1.0, 1.0, 0.1, 2, 3,
                                                                    precision=pr))
    err = rel(xg, ref.x)
    print(f"tall detector {prec}: rel L2 vs FP64 oracle {err:.2e}")
    assert rep["inner_done"] == 6 and rep["breakdown"] == 0
    assert err <= (SOLVE_TOL if prec == "fp32" else 1e-3)
    np.testing.assert_allclose(rep["phibar"], ref.phibar,
                               rtol=SOLVE_TOL if prec == "fp32" else 1e-3)


@pytest.mark.parametrize("prec", ["fp32", "f16"])
def test_solve_with_adjoint_view_chunks_same_bits(lib, prec):
    """A whole solve with A^T in chunks of 2 views (the 16-bit u-hat path for the
    mixed form on this geometry) returns the bits of the automatic choice."""
    import torch
    rng = np.random.default_rng(23)
    gg = lib.Geometry.from_dict(TALL)
    b = dev(rng.uniform(size=gg.proj_shape) * 5.0)
    xp = dev(rng.uniform(size=gg.vol_shape))
    pr = {"fp32": lib.PREC_FP32, "f16": lib.PREC_MIXED_F16_ADJ16}[prec]
    p = lib.SolveParams(1.0, 1.0, 0.1, 2, 3, precision=pr)
    outs = []
    for v in (0, 2):
        gg.set_back_views(v)
        x, rep = lib.solve(gg, b, xp, xp.clone(), p)
        assert rep["inner_done"] == 6
        outs.append(x)
    assert torch.equal(outs[0], outs[1])


def test_many_partials_against_oracle(orc, lib):
    """A volume whose stencil partials (20 480) take the two-stage reduction
    (k_psum, then k_red), as the benchmark sizes do: FP32 and mixed BF16 solves
    against the FP64 oracle."""
    rng = np.random.default_rng(29)
    d = dict(nx=128, ny=128, nz=320, vx=1.0, vy=1.0, vz=1.0, nu=128, nv=300, du=1.6, dv=1.6,
             dso=300.0, dsd=500.0, n_views=12)
    og = orc.Geometry.from_dict(d)
    xp = rng.uniform(size=og.vol_shape).astype(np.float32).astype(np.float64)
    xt = xp + 0.3 * (rng.uniform(size=og.vol_shape) > 0.95)
    b = orc.forward(og, xt).astype(np.float32).astype(np.float64)
    ref = orc.irn_piccs(og, b, xp, xp, 0.5, 1.5, 0.2, 2, 3)
    xg, rep = _gpu_solve(lib, d, b, xp, xp, lib.SolveParams(0.5, 1.5, 0.2, 2, 3))
    assert rep["inner_done"] == 6 and rep["breakdown"] == 0
    assert rel(xg, ref.x) <= SOLVE_TOL
    np.testing.assert_allclose(rep["phibar"], ref.phibar, rtol=SOLVE_TOL)
    xm, _ = _gpu_solve(lib, d, b, xp, xp,
                       lib.SolveParams(0.5, 1.5, 0.2, 2, 3, precision=lib.PREC_MIXED_BF16))
    assert rel(xm, ref.x) <= 1e-3


def test_mixed_forms_on_ragged_geometry(orc, lib):
    rng = np.random.default_rng(19)
    d = dict(nx=21, ny=19, nz=17, vx=1.0, vy=1.0, vz=1.0, nu=37, nv=150, du=1.1, dv=0.45,
             dso=80.0, dsd=130.0, n_views=13)
    og = orc.Geometry.from_dict(d)
    xp = rng.uniform(size=og.vol_shape).astype(np.float32).astype(np.float64)
    xt = xp + 0.3 * (rng.uniform(size=og.vol_shape) > 0.9)
    b = orc.forward(og, xt).astype(np.float32).astype(np.float64)
    ref = orc.irn_piccs(og, b, xp, xp, 0.5, 1.5, 0.2, 2, 4)
    for pr in (lib.PREC_MIXED_BF16, lib.PREC_MIXED_F16):
        xg, _ = _gpu_solve(lib, d, b, xp, xp, lib.SolveParams(0.5, 1.5, 0.2, 2, 4, precision=pr))
        assert rel(xg, ref.x) <= 1e-3


# ---------------------------------------------------------------- IRN-PIPLE

def test_c1_irn_piple_parity(orc, lib):
    """Third block lambda I, right-hand side lambda x_p (eq. seq_W_2)."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piple(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"],
                        sp["n_inner"])
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], sp["n_outer"], sp["n_inner"],
                        method=lib.METHOD_PIPLE)
    xg, rep = _gpu_solve(lib, d, b, prior, prior, p)
    assert rep["inner_done"] == sp["n_outer"] * sp["n_inner"] and rep["breakdown"] == 0
    assert rel(xg, ref.x) <= SOLVE_TOL
    np.testing.assert_allclose(rep["phibar"], ref.phibar, rtol=SOLVE_TOL)
    assert np.linalg.norm(xg - cur) < np.linalg.norm(prior - cur)


def test_piple_and_piccs_agree_without_the_prior_term(orc, lib):
    """lambda = 0 leaves IRN-TV in both methods: identical results."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    x1, r1 = _gpu_solve(lib, d, b, prior, prior, lib.SolveParams(sp["alpha"], 0.0, sp["tau"], 2, 4))
    x2, r2 = _gpu_solve(lib, d, b, prior, prior,
                        lib.SolveParams(sp["alpha"], 0.0, sp["tau"], 2, 4,
                                        method=lib.METHOD_PIPLE))
    assert np.array_equal(x1, x2)
    assert r1["phibar"] == r2["phibar"]


def test_piple_on_ragged_geometry_and_mixed(orc, lib):
    rng = np.random.default_rng(29)
    d = dict(nx=21, ny=19, nz=17, vx=1.0, vy=1.0, vz=1.0, nu=37, nv=150, du=1.1, dv=0.45,
             dso=80.0, dsd=130.0, n_views=13)
    og = orc.Geometry.from_dict(d)
    xp = rng.uniform(size=og.vol_shape).astype(np.float32).astype(np.float64)
    xt = xp + 0.3 * (rng.uniform(size=og.vol_shape) > 0.9)
    b = orc.forward(og, xt).astype(np.float32).astype(np.float64)
    ref = orc.irn_piple(og, b, xp, xp, 0.5, 1.5, 0.2, 2, 4)
    xg, _ = _gpu_solve(lib, d, b, xp, xp,
                       lib.SolveParams(0.5, 1.5, 0.2, 2, 4, method=lib.METHOD_PIPLE))
    assert rel(xg, ref.x) <= SOLVE_TOL
    for pr in (lib.PREC_MIXED_BF16, lib.PREC_MIXED_F16):
        xg, _ = _gpu_solve(lib, d, b, xp, xp,
                           lib.SolveParams(0.5, 1.5, 0.2, 2, 4, precision=pr,
                                           method=lib.METHOD_PIPLE))
        assert rel(xg, ref.x) <= 1e-3


def test_zero_data_breaks_down_immediately(orc, lib):
    """b = 0 from x_0 = x_p = 0: the first beta is 0, every outer step stops at
    once (breakdown), x stays 0 -- as in the oracle."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    z = np.zeros(og.vol_shape)
    zb = np.zeros(og.proj_shape)
    ref = orc.irn_piccs(og, zb, z, z, sp["alpha"], sp["lam"], sp["tau"], 2, 3)
    assert ref.breakdown and not np.any(ref.x)
    xg, rep = _gpu_solve(lib, d, zb, z, z, lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], 2, 3))
    assert not np.any(xg)
    assert rep["inner_done"] == 0 and rep["breakdown"] == 2 and rep["outer_done"] == 2


def test_full_size_lsqr_residual_estimate(lib):
    """256^3 / 90 views / 512^2, the benchmarked launch shape.  With alpha = lambda
    = 0 one outer step is plain LSQR, whose phibar_k equals ||b - A x_k|| in exact
    arithmetic and never grows (Sec. 2.2.2).  After 10 steps the device's estimate
    must match the residual recomputed with one more forward projection (float64
    norm) to 1e-5 (float32 vectors drift by ~1e-7 here): a property that holds at
    any size, so no oracle solve is needed."""
    import torch
    from paper_2509_08574_amd import synth
    gg = lib.Geometry.from_dict(synth.geometry("c2"))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    xt = torch.rand(gg.vol_shape, device="cuda", generator=gen)
    b = lib.forward(gg, xt)
    b += 0.01 * b.mean() * torch.randn(b.shape, device="cuda", generator=gen)
    x = torch.zeros_like(xt)
    x, rep = lib.solve(gg, b, torch.zeros_like(xt), x, lib.SolveParams(0.0, 0.0, 0.1, 1, 10))
    ph = np.array(rep["phibar"])
    assert rep["inner_done"] == 10 and rep["outer_done"] == 1 and rep["breakdown"] == 0
    assert np.all(np.diff(ph) <= 0.0)
    assert ph[-1] < 0.5 * ph[0]
    true = float(torch.linalg.norm((b - lib.forward(gg, x)).double()))
    assert abs(ph[-1] - true) <= 1e-5 * true


def test_reorth_matches_oracle(orc, lib):
    """reorth = 1: v reorthogonalised by classical Gram-Schmidt applied twice
    against the outer step's earlier v's (reading R18), as the oracle's option."""
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], 2, 8,
                        reorth=True)
    p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], 2, 8, reorth=1)
    xg, rep = _gpu_solve(lib, d, b, prior, prior, p)
    assert rep["inner_done"] == 16 and rep["breakdown"] == 0
    assert rel(xg, ref.x) <= SOLVE_TOL
    np.testing.assert_allclose(rep["phibar"], ref.phibar, rtol=SOLVE_TOL)


def test_reorth_long_plain_lsqr(orc, lib):
    """60 plain LSQR steps on a small ill-conditioned problem (12^3, 8 views;
    condition number of A ~ 8.7e3).  Here LSQR with float32 vectors leaves the
    float64 iterates after ~15 steps whatever the reorthogonalisation: an
    emulation on the oracle's dense A, every vector and product rounded to
    float32, gives the device's phibar to ~1e-3.  So the bar is relative: with
    reorth = 1 the device ends within 5e-3 of the oracle's reorthogonalised
    iterate, at least 3x closer than without it, and with a smaller residual."""
    d = dict(nx=12, ny=12, nz=12, vx=1.0, vy=1.0, vz=1.0, nu=24, nv=24, du=0.8, dv=0.8,
             dso=60.0, dsd=100.0, n_views=8)
    og = orc.Geometry.from_dict(d)
    rng = np.random.default_rng(3)
    b = orc.forward(og, rng.uniform(size=og.vol_shape)) + 0.01 * rng.normal(size=og.proj_shape)
    b = b.astype(np.float32).astype(np.float64)
    z = np.zeros(og.vol_shape)
    ref = orc.irn_piccs(og, b, z, z, 0.0, 0.0, 0.1, 1, 60, reorth=True)
    xr, rep_r = _gpu_solve(lib, d, b, z, z, lib.SolveParams(0.0, 0.0, 0.1, 1, 60, reorth=1))
    xp, rep_p = _gpu_solve(lib, d, b, z, z, lib.SolveParams(0.0, 0.0, 0.1, 1, 60))
    assert rep_r["inner_done"] == 60
    err_r, err_p = rel(xr, ref.x), rel(xp, ref.x)
    assert err_r <= 5e-3, err_r
    assert err_p >= 3 * err_r, (err_p, err_r)
    assert rep_r["phibar"][-1] < rep_p["phibar"][-1]


def test_reorth_mixed_precision(orc, lib):
    d, og, prior, cur, b, sp = c1_inputs(orc)
    ref = orc.irn_piccs(og, b, prior, prior, sp["alpha"], sp["lam"], sp["tau"], 2, 6,
                        reorth=True)
    for pr in (lib.PREC_MIXED_BF16, lib.PREC_MIXED_F16):
        p = lib.SolveParams(sp["alpha"], sp["lam"], sp["tau"], 2, 6, precision=pr, reorth=1)
        xg, _ = _gpu_solve(lib, d, b, prior, prior, p)
        assert rel(xg, ref.x) <= 1e-3
