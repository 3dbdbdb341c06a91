"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Each case prints its name before running so that a failing GPU step can be
identified from the log.  Tolerance for float32 (and split-bf16) results is
the relative L2 bound 1e-5 of the FP64 oracle (over the whole output, complex
entries counted as two reals), evaluated on the oracle applied to the same
float32-rounded input.
"""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from _util import ensure_built, per_degree_errors, rel_l2

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _record(name, payload):
    """Keep per-degree error profiles as JSON when SHT_TEST_RECORD_DIR is set
    (the GPU log keeps only the test outcome)."""
    d = os.environ.get("SHT_TEST_RECORD_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, name + ".json"), "w") as fh:
            json.dump(payload, fh)


# Per-degree bounds at 721 x 1440, lmax 720 (band-limited red spectrum
# a_lm ~ 1/(l+1) plus the 1e-3 white-noise probe).  A rounding error of
# relative size e in the products spreads over all (l, m) about evenly,
# while the energy of degree l falls like 1/(l+1); the per-degree rel-L2
# can therefore grow with l, up to ~ 3.6 e at l = 719 (sum over l of
# 2/(l+1) ~ 13 per field over 259,560 coefficients).  e is ~1e-7 for
# float32 and ~2.5e-6 (the two-plane table's representation error) for split
# bf16.  Measured worst degrees (MI355X): fp32 5.6e-7, split bf16 8.5e-6,
# three-term 3.4e-7; the rel-L2 bounds below are the model's value at
# l = 719 times ~4-5.  The max-error metric (largest |diff| of a degree over
# its largest |ref|, an extreme over 72 (l + 1) entries) measured 4.1e-6,
# 1.3e-4 and 3.2e-6; bounds ~4x those.
PER_DEGREE_TOL = {"fp32": 2e-6, "bf16x2": 4e-5, "bf16x3": 2e-6}
PER_DEGREE_MAX_TOL = {"fp32": 2e-5, "bf16x2": 5e-4, "bf16x3": 2e-5}


def _per_degree_check(tag, prec, got, ref):
    rel, mx = per_degree_errors(got, ref)
    _say(f"  {tag}: worst degree rel-L2 {rel.max():.3e} (l={int(rel.argmax())}), "
         f"worst degree max-err {mx.max():.3e} (l={int(mx.argmax())})")
    _record(f"per_degree_{tag}_{prec}", {"rel_l2": rel.tolist(), "max_err": mx.tolist()})
    if prec in PER_DEGREE_TOL:
        assert rel.max() <= PER_DEGREE_TOL[prec], (tag, float(rel.max()), int(rel.argmax()))
        assert mx.max() <= PER_DEGREE_MAX_TOL[prec], (tag, float(mx.max()), int(mx.argmax()))


def _say(*a):
    """Progress line: into pytest's captured output (shown with a failure)
    and, live, on the process's real stderr, so that a long test shows its
    steps while it runs."""
    print(*a, flush=True)
    print(*a, file=sys.__stderr__, flush=True)


@pytest.fixture(scope="module")
def pkg():
    ensure_built()
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2507_12144_amd as P
    return P


def _plan(P, nlat, nlon, lmax, mmax, grid, batch, channels, precision="fp32"):
    return P.Plan(dict(nlat=nlat, nlon=nlon, lmax=lmax, mmax=mmax, grid=grid, batch=batch, channels=channels),
                  precision=precision)


def _to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def _four_transforms(P, plan, shape, seed, prec_tol=TOL):
    """Run SHT, ISHT, SHT^T, ISHT^T on seeded inputs; return the four rel-L2s."""
    nlat, nlon, lmax, mmax, grid, B, C = shape
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((B, C, nlat, nlon)).astype(np.float32)
    a = synth.coefficients(seed + 1, B, C, lmax, mmax).astype(np.complex64)
    u64 = u.astype(np.float64)
    a64 = a.astype(np.complex128)
    du = _to_dev(u, torch.float32)
    da = _to_dev(a, torch.complex64)
    y = plan.sht(du).cpu().numpy()
    x = plan.isht(da).cpu().numpy()
    gx = plan.sht_T(da).cpu().numpy()
    gy = plan.isht_T(du).cpu().numpy()
    torch.cuda.synchronize()
    ref_y = oracle.sht(u64, lmax, mmax, grid)
    ref_x = oracle.isht(a64, nlat, nlon, grid)
    ref_gx = oracle.sht_T(a64, nlat, nlon, grid)
    ref_gy = oracle.isht_T(u64, lmax, mmax, grid)
    errs = (rel_l2(y, ref_y), rel_l2(x, ref_x), rel_l2(gx, ref_gx), rel_l2(gy, ref_gy))
    # exact structural zeros of the spectral outputs
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    for out in (y, gy):
        assert np.all(out[..., l < m] == 0)
        assert np.all(out[..., 0].imag == 0)
    return errs


SMALL = [
    # nlat, nlon, lmax, mmax, grid, batch, channels
    (32, 64, 32, 32, 1, 1, 4),       # the tiny Gauss-Legendre case
    (33, 64, 17, 17, 0, 1, 3),       # odd equiangular, equator ring, band limit
    (65, 128, 64, 40, 0, 2, 3),      # mmax < lmax
    (48, 96, 48, 48, 1, 1, 37),      # 74 columns: ragged second column tile
    (45, 90, 40, 40, 2, 1, 2),       # trapezoid weights, nlon = 2 * 3^2 * 5
    (181, 360, 180, 180, 0, 1, 5),   # 0.5 degree grid shape
    (16, 30, 10, 10, 1, 3, 1),       # nlon = 2 * 3 * 5
    (2, 2, 1, 1, 1, 1, 1),           # smallest legal transform
    (3, 4, 2, 2, 0, 1, 1),           # equator only besides the poles
    (9, 16, 30, 8, 1, 1, 2),         # lmax > nlat (aliased but well defined)
    (64, 128, 130, 64, 0, 1, 65),    # 130 columns, many row tiles per m
]


@pytest.mark.parametrize("shape", SMALL, ids=[f"{s[0]}x{s[1]}_L{s[2]}M{s[3]}_g{s[4]}_F{s[5]*s[6]}" for s in SMALL])
def test_small_parity_fp32(pkg, shape):
    _say("case", shape)
    plan = _plan(pkg, *shape)
    errs = _four_transforms(pkg, plan, shape, seed=3)
    _say("  rel-L2 sht/isht/sht_T/isht_T:", errs)
    assert max(errs) <= TOL, errs
    plan.close()


@pytest.mark.parametrize("nlat,grid", [(32, 1), (360, 1), (721, 0), (181, 0), (65, 2), (2, 1), (3, 0)])
def test_grid_matches_oracle(pkg, nlat, grid):
    _say("grid", nlat, grid)
    plan = _plan(pkg, nlat, 64, 2, 1, grid, 1, 1)
    x, w = plan.grid()
    _, xr, wr = oracle.grid(nlat, grid)
    np.testing.assert_allclose(x.numpy(), xr, atol=4e-16)
    np.testing.assert_allclose(w.numpy(), wr, rtol=1e-11, atol=1e-17)
    plan.close()


def test_full_size_equiangular_721_fp32(pkg):
    """721 x 1440, lmax = mmax = 720, 72 fields: the benchmark workload.
    Input: band-limited field (seed 0) plus a 1e-3 white-noise probe
    (seed 1), cast to float32; every output compared element by element."""
    nlat, nlon, L, B, C = 721, 1440, 720, 1, 72
    _say("full size 721x1440 fp32: building inputs")
    a = synth.coefficients(0, B, C, L, L)
    u = oracle.isht(a, nlat, nlon, 0) + synth.white_noise(1, (B, C, nlat, nlon))
    u32 = u.astype(np.float32)
    plan = _plan(pkg, nlat, nlon, L, L, 0, B, C)
    du = _to_dev(u32, torch.float32)
    y = plan.sht(du)
    x = plan.isht(y)
    gy = plan.isht_T(x)
    gx = plan.sht_T(gy)
    y, x, gy, gx = (t.cpu().numpy() for t in (y, x, gy, gx))
    _say("  oracle")
    # each stage's reference from the GPU stage's own (float32) input
    ref_y = oracle.sht(u32.astype(np.float64), L, L, 0)
    e1 = rel_l2(y, ref_y)
    _per_degree_check("sht", "fp32", y, ref_y)
    ref_x = oracle.isht(y.astype(np.complex128), nlat, nlon, 0)
    e2 = rel_l2(x, ref_x)
    ref_gy = oracle.isht_T(x.astype(np.float64), L, L, 0)
    e3 = rel_l2(gy, ref_gy)
    _per_degree_check("isht_T", "fp32", gy, ref_gy)
    ref_gx = oracle.sht_T(gy.astype(np.complex128), nlat, nlon, 0)
    e4 = rel_l2(gx, ref_gx)
    _say(f"  rel-L2 sht {e1:.3e} isht {e2:.3e} isht_T {e3:.3e} sht_T {e4:.3e}")
    assert max(e1, e2, e3, e4) <= TOL
    plan.close()


def _rdot(a, b):
    """Re sum conj(a) b in float64."""
    a, b = np.asarray(a).ravel(), np.asarray(b).ravel()
    if np.iscomplexobj(a) or np.iscomplexobj(b):
        return float(np.real(np.vdot(a.astype(np.complex128), b.astype(np.complex128))))
    return float(np.dot(a.astype(np.float64), b.astype(np.float64)))


@pytest.mark.parametrize("shape", [(33, 64, 17, 17, 0, 1, 3), (48, 96, 48, 48, 1, 2, 5), (181, 360, 180, 180, 0, 1, 8),
                                   (360, 720, 360, 360, 1, 4, 256)])
def test_gpu_adjoint_dot_products(pkg, shape):
    _say("dot", shape)
    nlat, nlon, lmax, mmax, grid, B, C = shape
    plan = _plan(pkg, *shape)
    rng = np.random.default_rng(21)
    u = rng.standard_normal((B, C, nlat, nlon)).astype(np.float32)
    g = synth.coefficients(22, B, C, lmax, mmax).astype(np.complex64)
    du, dg = _to_dev(u, torch.float32), _to_dev(g, torch.complex64)
    lhs = _rdot(plan.sht(du).cpu().numpy(), g)
    rhs = _rdot(u, plan.sht_T(dg).cpu().numpy())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs) + 1e-30) + 1e-6
    lhs = _rdot(plan.isht(dg).cpu().numpy(), u)
    rhs = _rdot(g, plan.isht_T(du).cpu().numpy())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs) + 1e-30) + 1e-6
    plan.close()


def test_autograd_functions(pkg):
    _say("autograd")
    P = pkg
    shape = (32, 64, 32, 32, 1, 2, 3)
    nlat, nlon, lmax, mmax, grid, B, C = shape
    plan = _plan(P, *shape)
    rng = np.random.default_rng(5)
    u = _to_dev(rng.standard_normal((B, C, nlat, nlon)), torch.float32).requires_grad_(True)
    r = rng.standard_normal((B, C, nlat, nlon))
    W = synth.mix_weights(4, lmax, C)
    loss = (P.ISHT.apply(P.ChannelMix.apply(P.SHT.apply(u, plan), _to_dev(W, torch.complex64), plan), plan)
            * _to_dev(r, torch.float32)).sum()
    loss.backward()
    ref = oracle.sht_T(oracle.channel_mix_T(oracle.isht_T(r, lmax, mmax, grid), W), nlat, nlon, grid)
    err = rel_l2(u.grad.cpu().numpy(), ref)
    _say("  grad rel-L2", err)
    assert err <= TOL
    plan.close()


MIX_SHAPES = [  # nlat, nlon, lmax, mmax, grid, batch, channels
    (24, 48, 24, 20, 1, 2, 37),      # one 64 x 64 tile per degree
    (48, 96, 40, 33, 1, 3, 130),     # three channel tiles (ragged), B * mmax > 64
]


@pytest.mark.parametrize("shape", MIX_SHAPES, ids=lambda s: f"B{s[5]}C{s[6]}L{s[2]}M{s[3]}")
def test_channel_mix_parity(pkg, shape):
    """Forward mix and mix^H against the oracle, every element."""
    _say("mix", shape)
    nlat, nlon, lmax, mmax, grid, B, C = shape
    plan = _plan(pkg, *shape)
    x = synth.coefficients(8, B, C, lmax, mmax)
    W = synth.mix_weights(9, lmax, C)
    dx, dW = _to_dev(x, torch.complex64), _to_dev(W, torch.complex64)
    y = plan.mix(dW, dx).cpu().numpy()
    yT = plan.mix(dW, dx, adjoint=True).cpu().numpy()
    e, eT = rel_l2(y, oracle.channel_mix(x, W)), rel_l2(yT, oracle.channel_mix_T(x, W))
    _say(f"  rel-L2 mix {e:.3e} mix^H {eT:.3e}")
    assert e <= TOL and eT <= TOL
    l = np.arange(lmax)[:, None]
    m = np.arange(mmax)[None, :]
    assert np.all(y[..., l < m] == 0) and np.all(yT[..., l < m] == 0)
    plan.close()


def test_channel_mix_parity_config4_sampled(pkg):
    """Forward mix and mix^H at the config-4 shape (4 x 256 channels, lmax =
    mmax = 360: four 64-channel tiles in each direction, 360 orders per
    degree) on the whole spectrum, compared with the oracle element by
    element at sampled degrees."""
    B, C, L = 4, 256, 360
    _say("mix 4x256 L360 (sampled degrees)")
    plan = _plan(pkg, 360, 720, L, L, 1, B, C)
    x = synth.coefficients(71, B, C, L, L).astype(np.complex64)
    W = synth.mix_weights(72, L, C).astype(np.complex64)
    dx, dW = _to_dev(x, torch.complex64), _to_dev(W, torch.complex64)
    y = plan.mix(dW, dx).cpu().numpy()
    yT = plan.mix(dW, dx, adjoint=True).cpu().numpy()
    for l in (0, 1, 63, 64, 65, 180, 359):
        xl = x[:, :, l:l + 1, :].astype(np.complex128)
        Wl = W[l:l + 1].astype(np.complex128)
        # the oracle on one degree: a [B, C, 1, mmax] spectrum with weight W_l
        mask = (np.arange(L) <= l)[None, None, None, :]
        ref = oracle.channel_mix(xl * mask, Wl)
        refT = oracle.channel_mix_T(xl * mask, Wl)
        e, eT = rel_l2(y[:, :, l:l + 1], ref), rel_l2(yT[:, :, l:l + 1], refT)
        _say(f"  l={l}: rel-L2 mix {e:.3e} mix^H {eT:.3e}")
        assert e <= TOL and eT <= TOL
    plan.close()


def test_bitwise_determinism(pkg):
    _say("determinism")
    shape = (181, 360, 180, 180, 0, 1, 9)
    plan = _plan(pkg, *shape)
    rng = np.random.default_rng(2)
    du = _to_dev(rng.standard_normal((1, 9, 181, 360)), torch.float32)
    y1 = plan.sht(du).clone()
    x1 = plan.isht(y1).clone()
    y2 = plan.sht(du)
    x2 = plan.isht(y2)
    assert torch.equal(y1, y2) and torch.equal(x1, x2)
    plan.close()


def test_python_argument_checks(pkg):
    plan = _plan(pkg, 16, 32, 16, 16, 1, 1, 2)
    with pytest.raises(ValueError):
        plan.sht(torch.zeros(1, 2, 16, 32, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        plan.sht(torch.zeros(1, 2, 16, 31, device="cuda"))
    with pytest.raises(ValueError):
        plan.isht(torch.zeros(1, 2, 16, 16, dtype=torch.complex64, device="cuda").transpose(-1, -2))
    with pytest.raises(ValueError):
        plan.sht(torch.zeros(1, 2, 16, 32))
    plan.close()


def test_non_default_stream(pkg):
    _say("stream")
    shape = (33, 64, 17, 17, 0, 1, 3)
    plan = _plan(pkg, *shape)
    rng = np.random.default_rng(4)
    u = rng.standard_normal((1, 3, 33, 64)).astype(np.float32)
    du = _to_dev(u, torch.float32)
    ref = plan.sht(du).clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        y = plan.sht(du)
    torch.cuda.current_stream().wait_stream(s)
    assert torch.equal(y, ref)
    plan.close()


MIX_GRAD_SHAPES = [  # batch, channels, lmax, mmax: ragged channel tiles, mmax < lmax, degenerate
    (2, 5, 7, 4), (3, 40, 33, 33), (2, 64, 65, 30), (1, 1, 1, 1)]


@pytest.mark.parametrize("shape", MIX_GRAD_SHAPES, ids=lambda s: "B{}C{}L{}M{}".format(*s))
def test_mix_weight_grad_parity(pkg, shape):
    """dW[l,c',c] = sum_{b, m <= l} g x^H of the per-degree channel mix
    against the FP64 oracle, every element (FP32 sums of at most B (l+1)
    products: rel-L2 within 1e-5)."""
    B, C, L, M = shape
    _say("mix weight grad", shape)
    nlon = 1 << (2 * M + 1).bit_length()  # a power of two >= 2 mmax + 2
    plan = _plan(pkg, 2 * L + 2, nlon, L, M, 1, B, C)
    g = synth.coefficients(41, B, C, L, M).astype(np.complex64)
    x = synth.coefficients(42, B, C, L, M).astype(np.complex64)
    dW = plan.mix_weight_grad(_to_dev(g, torch.complex64), _to_dev(x, torch.complex64)).cpu().numpy()
    ref = oracle.channel_mix_dW(g.astype(np.complex128), x.astype(np.complex128))
    err = rel_l2(dW, ref)
    _say(f"  rel-L2 {err:.3e}")
    assert err <= TOL
    plan.close()


def test_spectral_conv_block_gradients(pkg):
    """The spectral-convolution block L(x, W) = <r, ISHT(mix_W(SHT(x)))> on a
    Gauss 64 x 128 grid, lmax = mmax = 64, 2 x 48 channels, through
    torch.autograd: the weight gradient W.grad and the input gradient x.grad
    against the oracle's adjoint chain."""
    nlat, nlon, L, B, C = 64, 128, 64, 2, 48
    _say("spectral conv block 64x128 2x48")
    x = synth.grid_normal(51, (B, C, nlat, nlon)).astype(np.float32)
    r = synth.grid_normal(52, (B, C, nlat, nlon)).astype(np.float32)
    W = synth.mix_weights(53, L, C).astype(np.complex64)
    plan = _plan(pkg, nlat, nlon, L, L, 1, B, C)
    dx = _to_dev(x, torch.float32).requires_grad_(True)
    dW = _to_dev(W, torch.complex64).requires_grad_(True)
    out = pkg.ISHT.apply(pkg.ChannelMix.apply(pkg.SHT.apply(dx, plan), dW, plan), plan)
    (out * _to_dev(r, torch.float32)).sum().backward()
    r64, W64 = r.astype(np.float64), W.astype(np.complex128)
    gy = oracle.isht_T(r64, L, L, 1)
    ref_W = oracle.channel_mix_dW(gy, oracle.sht(x.astype(np.float64), L, L, 1))
    ref_x = oracle.sht_T(oracle.channel_mix_T(gy, W64), nlat, nlon, 1)
    eW, ex = rel_l2(dW.grad.cpu().numpy(), ref_W), rel_l2(dx.grad.cpu().numpy(), ref_x)
    _say(f"  W.grad rel-L2 {eW:.3e}, x.grad rel-L2 {ex:.3e}")
    assert eW <= TOL and ex <= TOL
    plan.close()


def test_mix_weight_grad_full_size_sampled(pkg):
    """Config-4 shape (4 x 256 channels, lmax = mmax = 360): the whole dW on
    the GPU, compared with the oracle at sampled degrees (first, second,
    middle, last) element by element."""
    B, C, L = 4, 256, 360
    _say("mix weight grad 4x256 L360 (sampled degrees)")
    plan = _plan(pkg, 360, 720, L, L, 1, B, C)
    g = synth.coefficients(61, B, C, L, L).astype(np.complex64)
    x = synth.coefficients(62, B, C, L, L).astype(np.complex64)
    dW = plan.mix_weight_grad(_to_dev(g, torch.complex64), _to_dev(x, torch.complex64)).cpu().numpy()
    degrees = [0, 1, 180, 359]
    ref = oracle.channel_mix_dW(g.astype(np.complex128), x.astype(np.complex128), degrees=degrees)
    for i, l in enumerate(degrees):
        err = rel_l2(dW[l], ref[i])
        _say(f"  l={l}: rel-L2 {err:.3e}")
        assert err <= TOL
    assert np.all(np.isfinite(dW))
    plan.close()


def test_differentiation_chain_gauss_360(pkg):
    """Gauss-Legendre 360 x 720, lmax = mmax = 360, batch 4 x 256 channels:
    L(x) = <r, ISHT(mix_W(SHT(x)))> with per-degree complex weights W_l
    (256 x 256, Re/Im ~ N(0, 1/512)).  Checked: the forward output against
    the oracle's forward chain; the GPU gradient (hand-written adjoint kernels
    through torch.autograd) against the FP64 oracle's adjoint chain (element
    by element); and against FP64 central differences (h = 1e-3) along 64
    random directions.  L is linear, so [L(x + h v) - L(x - h v)] / 2h =
    L(v) exactly.  60 directions are drawn on one field (b, c) each; their
    L(v) = <ISHT^T r_b, mix_W(SHT v)> takes the oracle's forward SHT and
    mix of the direction and the oracle's (separately pinned) ISHT adjoint of
    the cotangent.  4 directions span a whole ensemble member and go through
    the oracle's forward chain literally, and one more spans the whole input,
    evaluated at x + h v and x - h v."""
    P = pkg
    nlat, nlon, L, B, C = 360, 720, 360, 4, 256
    _say("chain 360x720 4x256: inputs")
    a = synth.coefficients(0, B, C, L, L)
    x = oracle.isht(a, nlat, nlon, 1).astype(np.float32)       # band-limited (seed 0)
    W = synth.mix_weights(4, L, C).astype(np.complex64)         # seed 4
    r = synth.grid_normal(3, (B, C, nlat, nlon)).astype(np.float32)  # cotangent (seed 3)
    plan = _plan(P, nlat, nlon, L, L, 1, B, C)
    dx = _to_dev(x, torch.float32).requires_grad_(True)
    dW = _to_dev(W, torch.complex64)
    dr = _to_dev(r, torch.float32)
    out = P.ISHT.apply(P.ChannelMix.apply(P.SHT.apply(dx, plan), dW, plan), plan)
    loss = (out * dr).sum()
    loss.backward()
    out_gpu = out.detach().cpu().numpy()
    g_gpu = dx.grad.cpu().numpy().astype(np.float64)
    W64, r64 = W.astype(np.complex128), r.astype(np.float64)

    def chain(u):
        return oracle.isht(oracle.channel_mix(oracle.sht(u, L, L, 1), W64), nlat, nlon, 1)

    _say("  oracle forward chain")
    e_out = rel_l2(out_gpu, chain(x.astype(np.float64)))
    _say(f"  forward output rel-L2 {e_out:.3e}")
    assert e_out <= TOL
    _say("  oracle adjoint chain")
    R = oracle.isht_T(r64, L, L, 1)                            # [B, C, L, L]
    g_ref = oracle.sht_T(oracle.channel_mix_T(R, W64), nlat, nlon, 1)
    e = rel_l2(g_gpu, g_ref)
    _say(f"  grad rel-L2 vs oracle adjoint {e:.3e}")
    assert e <= TOL
    gn = np.linalg.norm(g_ref)
    del g_ref
    rng = np.random.default_rng(2)
    worst = 0.0
    for i in range(60):
        b, c = int(rng.integers(B)), int(rng.integers(C))
        v = rng.standard_normal((nlat, nlon))
        s1 = oracle.sht(v[None, None], L, L, 1)[0, 0]          # [L, L]
        # mix_W of a spectrum that is s1 in channel c and 0 elsewhere:
        # channel c' holds W_l[c', c] s1[l, m]
        y = W64[:, :, c].T[:, :, None] * s1[None, :, :]        # [C', L, L]
        fd = float(np.sum(np.real(np.conj(R[b]) * y)))
        d = abs(fd - float(np.sum(g_gpu[b, c] * v))) / (gn * np.linalg.norm(v))
        worst = max(worst, d)
    _say(f"  60 single-field directions: worst rel err {worst:.3e}")
    assert worst <= TOL
    del R
    for i in range(4):
        v = rng.standard_normal((1, C, nlat, nlon))
        fd = float(np.sum(r64[i:i + 1] * chain(v)))
        d = abs(fd - float(np.sum(g_gpu[i:i + 1] * v))) / (gn * np.linalg.norm(v))
        _say(f"  member-{i} direction through the forward chain: rel err {d:.3e}")
        assert d <= TOL

    def lossf(u):
        return float(np.sum(r64 * chain(u)))

    h = 1e-3
    x64 = x.astype(np.float64)
    v = np.random.default_rng(11).standard_normal(x.shape)
    fd = (lossf(x64 + h * v) - lossf(x64 - h * v)) / (2 * h)
    d = abs(fd - np.sum(g_gpu * v)) / (gn * np.linalg.norm(v))
    _say(f"  literal central difference, full-support direction: rel err {d:.3e}")
    assert d <= TOL
    plan.close()


def test_plan_allocation_failures_are_clean(pkg):
    """SHT_TEST_FAIL_ALLOC=n fails the n-th device allocation of a plan build:
    every n up to the build's allocation count must give SHT_ERR_OUT_OF_MEMORY
    and free what the build had allocated (device memory back to its level
    before); a build without the hook then succeeds and computes."""
    _say("allocation failure injection")
    desc = dict(nlat=181, nlon=360, lmax=180, mmax=180, grid="equiangular", batch=1, channels=40)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    n = 0
    try:
        while True:
            n += 1
            os.environ["SHT_TEST_FAIL_ALLOC"] = str(n)
            try:
                plan = pkg.Plan(desc)
            except pkg.ShtError as e:
                assert e.status == 3, (n, e)          # SHT_ERR_OUT_OF_MEMORY
                continue
            plan.close()                               # n is past the build's last allocation
            break
    finally:
        os.environ.pop("SHT_TEST_FAIL_ALLOC", None)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    _say(f"  {n - 1} allocations failed in turn; device free memory before {free0} after {free1}")
    assert n > 5
    assert free0 - free1 < 4 << 20, (free0, free1)
    plan = pkg.Plan(desc)
    u = torch.randn(1, 40, 181, 360, device="cuda")
    y = plan.sht(u)
    assert torch.isfinite(torch.view_as_real(y)).all()
    plan.close()


# tolerance per precision form: split bf16 meets the 1e-5 target, the
# three-term split reaches float32 level, plain bf16 is reported at ~3e-3
PREC_TOL = {"bf16": 1e-2, "bf16x2": 1e-5, "bf16x3": 1e-6}


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "bf16x3"])
@pytest.mark.parametrize("shape", [SMALL[0], SMALL[2], SMALL[3], SMALL[5], SMALL[7], SMALL[10]],
                         ids=lambda s: f"{s[0]}x{s[1]}_L{s[2]}M{s[3]}_F{s[5]*s[6]}" if isinstance(s, tuple) else s)
def test_small_parity_bf16_forms(pkg, shape, prec):
    _say("case", prec, shape)
    plan = _plan(pkg, *shape, precision=prec)
    errs = _four_transforms(pkg, plan, shape, seed=5)
    _say("  rel-L2 sht/isht/sht_T/isht_T:", errs)
    assert max(errs) <= PREC_TOL[prec], errs
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "bf16x3"])
def test_full_size_equiangular_721_bf16_forms(pkg, prec):
    """721 x 1440, lmax 720, 72 fields in each bf16 form: relative L2 of all
    four transforms (SHT -> ISHT -> ISHT^T -> SHT^T, each against the oracle
    applied to the GPU stage's own input) and the per-degree errors of the
    spectral outputs."""
    nlat, nlon, L, B, C = 721, 1440, 720, 1, 72
    _say(f"full size 721x1440 {prec}")
    a = synth.coefficients(0, B, C, L, L)
    u32 = (oracle.isht(a, nlat, nlon, 0) + synth.white_noise(1, (B, C, nlat, nlon))).astype(np.float32)
    plan = _plan(pkg, nlat, nlon, L, L, 0, B, C, precision=prec)
    y = plan.sht(_to_dev(u32, torch.float32))
    x = plan.isht(y)
    gy = plan.isht_T(x)
    gx = plan.sht_T(gy)
    y, x, gy, gx = (t.cpu().numpy() for t in (y, x, gy, gx))
    _say("  oracle")
    ref_y = oracle.sht(u32.astype(np.float64), L, L, 0)
    e1 = rel_l2(y, ref_y)
    _per_degree_check("sht", prec, y, ref_y)
    del ref_y
    e2 = rel_l2(x, oracle.isht(y.astype(np.complex128), nlat, nlon, 0))
    ref_gy = oracle.isht_T(x.astype(np.float64), L, L, 0)
    e3 = rel_l2(gy, ref_gy)
    _per_degree_check("isht_T", prec, gy, ref_gy)
    del ref_gy
    e4 = rel_l2(gx, oracle.sht_T(gy.astype(np.complex128), nlat, nlon, 0))
    _say(f"  {prec}: rel-L2 sht {e1:.3e} isht {e2:.3e} isht_T {e3:.3e} sht_T {e4:.3e}")
    _record(f"full_size_{prec}", {"sht": e1, "isht": e2, "isht_T": e3, "sht_T": e4})
    assert max(e1, e2, e3, e4) <= PREC_TOL[prec], (e1, e2, e3, e4)
    plan.close()


BATCH_MIX = [
    # segments of one plan: every ring padding (kpad 64 .. 384) and DFT path
    (33, 64, 17, 17, 0, 1, 3),
    (45, 90, 40, 40, 2, 1, 2),       # generic-radix ring DFT
    (181, 360, 180, 180, 0, 1, 5),   # kpad 128
    (32, 64, 32, 32, 1, 2, 2),
    (361, 720, 360, 360, 0, 1, 2),   # kpad 192
    (401, 720, 300, 300, 1, 1, 1),   # kpad 256 (Gauss, 201 northern rings)
    (721, 1440, 720, 720, 0, 1, 1),  # kpad 384
]


def _batched_io(P, plan, shapes, seed):
    """Flat inputs of a multi-segment plan, filled segment by segment."""
    rng = np.random.default_rng(seed)
    u = np.zeros(plan.grid_elems, np.float32)
    a = np.zeros(plan.spec_elems, np.complex64)
    parts = []
    for i, (nlat, nlon, lmax, mmax, grid, B, C) in enumerate(shapes):
        go, so = plan.segment(i)
        ui = rng.standard_normal((B, C, nlat, nlon)).astype(np.float32)
        ai = synth.coefficients(seed + 7 + i, B, C, lmax, mmax).astype(np.complex64)
        u[go:go + ui.size] = ui.ravel()
        a[so:so + ai.size] = ai.ravel()
        parts.append((go, so, ui, ai))
    return u, a, parts


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x2", "bf16x3"])
def test_batched_uneven_segments(pkg, prec):
    """One plan over segments of every ring padding and both ring-DFT paths:
    each segment's four transforms against the oracle, and bitwise equal to
    a single-segment plan of the same shape (the same kernel body runs)."""
    _say("batched plan over", len(BATCH_MIX), "segments", prec)
    tol = TOL if prec == "fp32" else PREC_TOL[prec]
    plan = _multi_plan(pkg, BATCH_MIX, prec)
    u, a, parts = _batched_io(pkg, plan, BATCH_MIX, seed=21)
    du, da = _to_dev(u, torch.float32), _to_dev(a, torch.complex64)
    outs = [plan.sht(du).cpu().numpy(), plan.isht(da).cpu().numpy(), plan.sht_T(da).cpu().numpy(),
            plan.isht_T(du).cpu().numpy()]
    for i, (shape, (go, so, ui, ai)) in enumerate(zip(BATCH_MIX, parts)):
        nlat, nlon, lmax, mmax, grid, B, C = shape
        _say("  segment", i, shape)
        ng, ns = ui.size, ai.size
        y = outs[0][so:so + ns].reshape(ai.shape)
        x = outs[1][go:go + ng].reshape(ui.shape)
        gx = outs[2][go:go + ng].reshape(ui.shape)
        gy = outs[3][so:so + ns].reshape(ai.shape)
        u64, a64 = ui.astype(np.float64), ai.astype(np.complex128)
        errs = (rel_l2(y, oracle.sht(u64, lmax, mmax, grid)), rel_l2(x, oracle.isht(a64, nlat, nlon, grid)),
                rel_l2(gx, oracle.sht_T(a64, nlat, nlon, grid)), rel_l2(gy, oracle.isht_T(u64, lmax, mmax, grid)))
        _say("    rel-L2 sht/isht/sht_T/isht_T:", errs)
        assert max(errs) <= tol, (shape, errs)
        single = _plan(pkg, *shape, precision=prec)
        dui, dai = _to_dev(ui, torch.float32), _to_dev(ai, torch.complex64)
        for got, ref in ((y, single.sht(dui)), (x, single.isht(dai)), (gx, single.sht_T(dai)),
                         (gy, single.isht_T(dui))):
            assert np.array_equal(got, ref.cpu().numpy()), shape
        single.close()
    plan.close()


GRAPH_SEGS = [(33, 64, 17, 17, 0, 1, 3), (181, 360, 180, 180, 0, 2, 3), (32, 64, 32, 32, 1, 1, 2)]


def _multi_plan(P, shapes, precision="fp32"):
    return P.Plan([dict(nlat=s[0], nlon=s[1], lmax=s[2], mmax=s[3], grid=s[4], batch=s[5], channels=s[6])
                   for s in shapes], precision=precision)


def _segment_mask(plan, shapes, spectral):
    """True on the entries of the segments (the alignment gaps between
    segments are never written)."""
    n = plan.spec_elems if spectral else plan.grid_elems
    mask = np.zeros(n, bool)
    for i, (nlat, nlon, lmax, mmax, grid, B, C) in enumerate(shapes):
        go, so = plan.segment(i)
        off, size = (so, B * C * lmax * mmax) if spectral else (go, B * C * nlat * nlon)
        mask[off:off + size] = True
    return mask


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_graph_replay_matches_eager(pkg, prec):
    """The fwd+bwd chain SHT -> ISHT -> ISHT^T -> SHT^T captured as one HIP
    graph; several replays, with eager work and synchronisation between them,
    each equal bit for bit to the eager chain (float32: staged analysis
    output, the spectrum transpose in the graph; split bf16: both directions
    staged, the staging kernel in the graph too)."""
    _say("graph replay over", GRAPH_SEGS, prec)
    plan = _multi_plan(pkg, GRAPH_SEGS, prec)
    u_h, _, _ = _batched_io(pkg, plan, GRAPH_SEGS, seed=5)
    u = _to_dev(u_h, torch.float32)
    y = plan.sht(u)
    x = plan.isht(y)
    gy = plan.isht_T(x)
    gx = plan.sht_T(gy)
    ref = [t.cpu().numpy() for t in (y, x, gy, gx)]
    ys, xs, gys, gxs = (torch.empty_like(t) for t in (y, x, gy, gx))
    g = plan.graph([("sht", u, ys), ("isht", ys, xs), ("isht_T", xs, gys), ("sht_T", gys, gxs)])
    other = torch.randn_like(u)
    masks = [_segment_mask(plan, GRAPH_SEGS, sp) for sp in (True, False, True, False)]
    for rep in range(4):
        for t in (ys, xs, gys, gxs):
            t.zero_()
        g.launch()
        torch.cuda.synchronize()
        for got, r, mk in zip((ys, xs, gys, gxs), ref, masks):
            assert np.array_equal(got.cpu().numpy()[mk], r[mk]), rep
        plan.sht(other)          # eager work on the same plan between replays
        (other * 2).sum().item()
        torch.cuda.synchronize()
    with pytest.raises(pkg.ShtError):
        plan.close()             # graphs must go first
    g.close()
    plan.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16x2"])
def test_tune_parity_and_cache(pkg, tmp_path, prec):
    """Every tuning candidate must reproduce the default schedule's outputs
    bit for bit (checked inside sht_plan_tune); the chosen schedule gives the
    same outputs as before tuning, and the cached choice is reused."""
    _say("tune", prec)
    plan = _multi_plan(pkg, GRAPH_SEGS, prec)
    u_h, a_h, _ = _batched_io(pkg, plan, GRAPH_SEGS, seed=9)
    u, a = _to_dev(u_h, torch.float32), _to_dev(a_h, torch.complex64)
    before = [plan.sht(u).cpu().numpy(), plan.isht(a).cpu().numpy()]
    cache = tmp_path / "tune.txt"
    choice, ms = plan.tune(cache)
    _say("  chosen", choice, "ms", ms)
    assert ms > 0
    after = [plan.sht(u).cpu().numpy(), plan.isht(a).cpu().numpy()]
    masks = [_segment_mask(plan, GRAPH_SEGS, True), _segment_mask(plan, GRAPH_SEGS, False)]
    for b, c, mk in zip(before, after, masks):
        assert np.array_equal(b[mk], c[mk])
    plan2 = _multi_plan(pkg, GRAPH_SEGS, prec)
    choice2, ms2 = plan2.tune(cache)
    assert (choice2, ms2) == (choice, -1.0)
    assert np.array_equal(plan2.sht(u).cpu().numpy()[masks[0]], before[0][masks[0]])
    plan.close()
    plan2.close()


@pytest.mark.parametrize("shape", [(721, 1440, 720, 720, 0, 1, 72), (360, 720, 360, 360, 1, 4, 40),
                                   (181, 360, 180, 180, 0, 1, 37)],
                         ids=lambda s: f"{s[0]}x{s[1]}_F{s[5] * s[6]}")
def test_field_groups_per_workgroup_are_bitwise_equal(pkg, shape):
    """The float32 kernels with 2, 3 and 4 field groups per workgroup and
    with the analysis output staged (order-major tiles + spectrum transpose)
    or stored directly (tuning choices) give the same bits for all four
    transforms, also with a ragged last column chunk."""
    _say("schedules", shape)
    nlat, nlon, L, M, grid, B, C = shape
    plan = _plan(pkg, *shape)
    u = _to_dev(synth.grid_normal(31, (B, C, nlat, nlon)), torch.float32)
    a = _to_dev(synth.coefficients(32, B, C, L, M), torch.complex64)
    ref = None
    for staged in (0, 1, 2, 3):
        for ncb in (2, 3, 4):
            plan.set_schedule(8, 0, ncb, staged)
            assert plan.schedule() == (8, 0, ncb, staged)
            outs = [plan.sht(u), plan.isht(a), plan.sht_T(a), plan.isht_T(u)]
            if ref is None:
                ref = outs
            else:
                for o, r in zip(outs, ref):
                    assert torch.equal(o, r), (ncb, staged)
    plan.close()


@pytest.mark.parametrize("prec", ["bf16", "bf16x2", "bf16x3"])
def test_staged_analysis_bitwise_equal_bf16_forms(pkg, prec):
    """Staged and direct analysis output and synthesis input of the bf16
    forms, bitwise, on a multi-segment plan (every ring padding, odd mmax,
    mmax < lmax)."""
    shapes = [(33, 64, 17, 17, 0, 1, 3), (65, 128, 64, 41, 0, 2, 3), (181, 360, 180, 180, 0, 1, 5),
              (721, 1440, 720, 720, 0, 1, 2)]
    _say("staged bf16", prec)
    plan = _multi_plan(pkg, shapes, prec)
    u_h, _, _ = _batched_io(pkg, plan, shapes, seed=33)
    u = _to_dev(u_h, torch.float32)
    mask = _segment_mask(plan, shapes, True)
    a_h = np.zeros(plan.spec_elems, np.complex64)
    for i, (nlat, nlon, lmax, mmax, grid, B, C) in enumerate(shapes):
        _, so = plan.segment(i)
        ai = synth.coefficients(34 + i, B, C, lmax, mmax).astype(np.complex64)
        a_h[so:so + ai.size] = ai.ravel()
    a = _to_dev(a_h, torch.complex64)
    gmask = _segment_mask(plan, shapes, False)
    outs = []
    for staged in (0, 1, 2, 3):
        plan.set_schedule(8, 0, 2, staged)
        outs.append((plan.sht(u).cpu().numpy()[mask], plan.isht_T(u).cpu().numpy()[mask],
                     plan.isht(a).cpu().numpy()[gmask], plan.sht_T(a).cpu().numpy()[gmask]))
    for o in outs[1:]:
        for x, r in zip(o, outs[0]):
            assert np.array_equal(x, r)
    plan.close()


def test_environment_switches(pkg, tmp_path):
    """SHT_AUTOTUNE=1 tunes every new plan (its choice lands in the
    SHT_TUNE_CACHE file); SHT_DEBUG=1 synchronises after every kernel and
    leaves the results unchanged."""
    _say("environment switches")
    shape = (33, 64, 17, 17, 0, 1, 3)
    u = _to_dev(synth.grid_normal(41, (1, 3, 33, 64)), torch.float32)
    plan = _plan(pkg, *shape)
    ref = plan.sht(u).cpu().numpy()
    plan.close()
    cache = tmp_path / "tune.txt"
    os.environ["SHT_AUTOTUNE"] = "1"
    os.environ["SHT_TUNE_CACHE"] = str(cache)
    os.environ["SHT_DEBUG"] = "1"
    try:
        plan = _plan(pkg, *shape)
        got = plan.sht(u).cpu().numpy()
        plan.close()
    finally:
        for k in ("SHT_AUTOTUNE", "SHT_TUNE_CACHE", "SHT_DEBUG"):
            os.environ.pop(k, None)
    assert cache.exists() and len(cache.read_text().splitlines()) == 1
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("prec", ["fp32", "bf16", "bf16x2", "bf16x3"])
def test_race_check_build_bitwise_equal(pkg, prec):
    """The race-check build libsht_debug.so (every barrier drains all memory
    counters and every Legendre stage ends with a drain and a workgroup
    barrier, so no copy, load or store of one stage overlaps another stage's
    work) gives the release library's outputs bit for bit: all four
    transforms, direct and staged spectra, a multi-segment plan with every
    ring padding, odd mmax and mmax < lmax, and the scores and mix kernels
    that use the same barriers."""
    path = os.path.join(os.path.dirname(pkg.__file__), "libsht_debug.so")
    assert os.path.exists(path), "libsht_debug.so is not built: python -m paper_2507_12144_amd.build debug"
    shapes = [(33, 64, 17, 17, 0, 1, 3), (65, 128, 64, 41, 0, 2, 3), (181, 360, 180, 180, 0, 1, 5),
              (90, 180, 90, 90, 1, 1, 20), (361, 720, 360, 360, 0, 1, 9)]
    _say("race-check build", prec)
    debug = pkg._lib.open_library(path)
    plans = [_multi_plan(pkg, shapes, prec),
             pkg.Plan([dict(nlat=s[0], nlon=s[1], lmax=s[2], mmax=s[3], grid=s[4], batch=s[5], channels=s[6])
                       for s in shapes], precision=prec, library=debug)]
    u_h, _, _ = _batched_io(pkg, plans[0], shapes, seed=51)
    u = _to_dev(u_h, torch.float32)
    a_h = np.zeros(plans[0].spec_elems, np.complex64)
    for i, (nlat, nlon, lmax, mmax, grid, B, C) in enumerate(shapes):
        _, so = plans[0].segment(i)
        ai = synth.coefficients(52 + i, B, C, lmax, mmax).astype(np.complex64)
        a_h[so:so + ai.size] = ai.ravel()
    a = _to_dev(a_h, torch.complex64)
    smask, gmask = _segment_mask(plans[0], shapes, True), _segment_mask(plans[0], shapes, False)
    outs = []
    for plan in plans:
        res = []
        for staged in (0, 3):
            plan.set_schedule(8, 0, 2, staged)
            res += [plan.sht(u).cpu().numpy()[smask], plan.isht_T(u).cpu().numpy()[smask],
                    plan.isht(a).cpu().numpy()[gmask], plan.sht_T(a).cpu().numpy()[gmask]]
        outs.append(res)
    for i, (d, r) in enumerate(zip(outs[1], outs[0])):
        assert np.array_equal(d, r), i
    for plan in plans:
        plan.close()
    if prec != "fp32":
        return
    # single-segment plans: the channel mix, its weight gradient and the
    # spectral CRPS with gradient (LDS-staged GEMM tiles and block sums)
    B, C, L = 2, 48, 40
    desc = dict(nlat=42, nlon=80, lmax=L, mmax=L, grid="gauss", batch=B, channels=C)
    p0, p1 = pkg.Plan(desc), pkg.Plan(desc, library=debug)
    g = torch.Generator(device="cuda").manual_seed(53)
    x = torch.randn((B, C, L, L), device="cuda", dtype=torch.complex64, generator=g)
    W = torch.randn((L, C, C), device="cuda", dtype=torch.complex64, generator=g)
    for f in (lambda p: p.mix(W, x), lambda p: p.mix(W, x, adjoint=True), lambda p: p.mix_weight_grad(x, x)):
        assert torch.equal(f(p0), f(p1))
    obs = x[0]
    l0, g0 = p0.spectral_crps(x, obs, grad=True)
    l1, g1 = p1.spectral_crps(x, obs, grad=True)
    assert torch.equal(l0, l1) and torch.equal(g0, g1)
    p0.close()
    p1.close()
