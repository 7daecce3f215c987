"""GPU parity of every hot-path operator against the oracle, element by
element, on seeded random inputs (FP64: relative 1e-12; FP32: 1e-5)."""
import numpy as np
import pytest

from gpu_util import Pair, small, to_dev, to_np, rel, torch_mod

pytestmark = pytest.mark.gpu

CASES = [
    dict(dim=2, n=3, level=1, order=4),            # ragged: S = 36
    dict(dim=2, n=5, level=2, order=8, seed=1),    # S = 100, A = 384
    dict(dim=3, n=3, level=1, order=6, seed=2),    # S = 216
    dict(dim=3, n=4, level=2, order=10, seed=3),   # S = 512, A = 384 (several GEMM tiles)
    # cones around an oblique axis (levels of 32, 50, 89 patches): octant
    # blocks of three reflections on level 1, of one (the x reflection) on
    # level 2, none on level 3, where the order-10 case takes the dense
    # product and the order-4 case the factored one (as does its level 2)
    dict(dim=3, n=3, level=1, order=10, seed=5, angular=(1, (0.3, 0.5, 0.81), 25.0, 2)),
    dict(dim=3, n=3, level=1, order=4, seed=6, angular=(1, (0.3, 0.5, 0.81), 25.0, 2)),
]


@pytest.fixture(scope="module", params=range(len(CASES)))
def pair(request):
    kw = dict(CASES[request.param])
    print("case", kw, flush=True)
    if "angular" in kw:
        from paper_2010_04559_amd import inputs
        base, axis, half, extra = kw.pop("angular")
        kw["angular"] = inputs.AngularSpec(base, axis, half, extra, True)
    return Pair(small(**kw))


def test_scatter_forms(pair):
    """Uniform meshes: every level >= 1 in octant-block form (3 reflected
    axes); the oblique cone's refined level has no reflection symmetry."""
    forms = pair.tr.scatter_forms
    assert forms[0] == ("dense", 0)
    if pair.prob.angular.extra_levels == 0:
        assert all(f == ("octant", 3) for f in forms[1:]), forms
        assert pair.tr.outer_axes == 3
    elif pair.prob.order == 10:
        assert forms[1:] == [("octant", 3), ("octant", 1), ("dense", 0)], forms
        assert pair.tr.outer_axes == 0
    else:
        assert forms[1:] == [("octant", 3), ("factored", 25), ("factored", 25)], forms
        assert pair.tr.outer_axes == 0


def _rand(n, seed):
    return np.random.default_rng(seed).standard_normal(n)


def test_sweep_fp64(pair):
    for l in range(pair.tr.nlev):
        lv = pair.level(l)
        g = _rand(lv.A * lv.grid.S, 10 + l)
        got = to_np(pair.tr.sweep(l, to_dev(g)))
        assert rel(got, lv.sweep(g)) < 1e-12, l


def test_sweep_adjoint_fp64(pair):
    for l in range(pair.tr.nlev):
        lv = pair.level(l)
        g = _rand(lv.A * lv.grid.S, 20 + l)
        got = to_np(pair.tr.sweep(l, to_dev(g), adjoint=True))
        assert rel(got, lv.sweep_T(g)) < 1e-12, l


def test_sweep_fp32(pair):
    torch = torch_mod()
    l = pair.tr.nlev - 1
    lv = pair.level(l)
    g = _rand(lv.A * lv.grid.S, 30)
    got = to_np(pair.tr.sweep(l, to_dev(g, torch.float32)))
    assert rel(got, lv.sweep(g)) < 2e-5


def test_scatter_levels_and_outer(pair):
    for l in range(pair.tr.nlev):
        lv = pair.level(l)
        x = _rand(lv.A * lv.grid.S, 40 + l)
        got = to_np(pair.tr.scatter(l, to_dev(x)))
        assert rel(got, lv.apply_S(x)) < 1e-12, l
    lv = pair.level(0, outer=True)
    x = _rand(lv.A * lv.grid.S, 50)
    got = to_np(pair.tr.scatter(pair.tr.nlev - 1, to_dev(x), outer=True))
    assert rel(got, lv.apply_S(x)) < 1e-12


def test_scatter_fp32(pair):
    torch = torch_mod()
    l = pair.tr.nlev - 1
    lv = pair.level(l)
    x = _rand(lv.A * lv.grid.S, 60)
    got = to_np(pair.tr.scatter(l, to_dev(x, torch.float32)))
    assert rel(got, lv.apply_S(x)) < 1e-5


def test_scatter_split_bf16(pair):
    """FP32 scatter with split-BF16 operands against the FP64 oracle.  Each
    product a b is formed as a_hi b_hi + a_hi b_lo + a_lo b_hi with
    |a - a_hi - a_lo| <= 2^-16 |a| (two round-to-nearest BF16 steps) and the
    dropped |a_lo b_lo| <= 2^-16 |a b|: at most 3 2^-16 = 4.6e-5 relative per
    term, plus FP32 accumulation; norm-wise over these random inputs the sum
    stays within 2e-4 (cancellation factor below 4)."""
    torch = torch_mod()
    for l in range(1, pair.tr.nlev):
        lv = pair.level(l)
        x = _rand(lv.A * lv.grid.S, 62 + l)
        got = to_np(pair.tr.scatter(l, to_dev(x, torch.float32), split_bf16=True))
        ref = lv.apply_S(x)
        assert rel(got, ref) < 2e-4, l
        # and it is really the split product, not plain FP32 (which is ~1e-7)
        assert rel(got, ref) > 1e-8, l


def test_apply(pair):
    lv = pair.level(0, outer=True)
    x = _rand(lv.A * lv.grid.S, 70)
    got = to_np(pair.tr.apply(to_dev(x)))
    assert rel(got, lv.apply_A(x)) < 1e-12


def test_transfers(pair):
    mg = pair.op.mg
    S = mg.grid.S
    for l in range(1, pair.tr.nlev):
        xc = _rand(mg.levels[l - 1].A * S, 80 + l)
        got = to_np(pair.tr.prolong(l, to_dev(xc)))
        assert rel(got, mg.prolong(l, xc)) < 1e-14
        xf = _rand(mg.levels[l].A * S, 90 + l)
        got = to_np(pair.tr.restrict(l, to_dev(xf)))
        assert rel(got, mg.restrict(l, xf)) < 1e-14


@pytest.mark.parametrize("nu", [1, 3])
def test_coarse_gauss_seidel(pair, nu):
    lv0 = pair.op.mg.levels[0]
    f = _rand(lv0.A * lv0.grid.S, 100 + nu)
    got = to_np(pair.tr.coarse_gs(to_dev(f), nu))
    assert rel(got, pair.op.mg.coarse_gs(f, nu)) < 1e-11
    got = to_np(pair.tr.coarse_gs(to_dev(f), nu, adjoint=True))
    assert rel(got, pair.op.mg.coarse_gs(f, nu, adjoint=True)) < 1e-11


def test_vcycle_fp64(pair):
    lv = pair.level(0, outer=True)
    r = _rand(lv.A * lv.grid.S, 110)
    got = to_np(pair.tr.vcycle(to_dev(r)))
    assert rel(got, pair.op.mg.vcycle(r)) < 1e-11
    got = to_np(pair.tr.vcycle(to_dev(r), adjoint=True))
    assert rel(got, pair.op.mg.vcycle(r, adjoint=True)) < 1e-11
    got = to_np(pair.tr.vcycle(to_dev(r), mode="sg"))
    assert rel(got, lv.sweep(r)) < 1e-12


def test_vcycle_mixed_precision(pair):
    lv = pair.level(0, outer=True)
    r = _rand(lv.A * lv.grid.S, 120)
    got = to_np(pair.tr.vcycle(to_dev(r), mode="mixed"))
    assert rel(got, pair.op.mg.vcycle(r)) < 1e-4


def test_rhs_and_detector(pair):
    prob = pair.prob
    got = to_np(pair.tr.rhs())
    assert rel(got, pair.op.rhs()) < 1e-13
    lo, hi = (0, 1, 0), (1, 2, 1)
    got = to_np(pair.tr.detector(lo, hi))
    assert rel(got, pair.op.outer.detector_weights(lo, hi)) < 1e-13


def test_determinism(pair):
    lv = pair.level(0, outer=True)
    r = to_dev(_rand(lv.A * lv.grid.S, 130))
    a = to_np(pair.tr.vcycle(r))
    b = to_np(pair.tr.vcycle(r))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("n", [(28, 28, 28), (64, 64, 20), (6, 5, 7), (2, 3, 9), (48, 10, 6), (7, 6, 4)])
def test_sweep_large_planes(n):
    """Planes of 588 and ~1280 cells (several cells per thread per plane),
    and grids of even and odd cell counts along x: with an even count the
    forward sweep runs over bricks of two x-adjacent cells (FP32 and FP64
    where the brick planes fit), with an odd one over cells."""
    from paper_2010_04559_amd import inputs
    torch = torch_mod()
    prob = inputs.small_problem(dim=3, n=4, level=0, order=2, seed=12)
    C = n[0] * n[1] * n[2]
    rng = np.random.default_rng(13)
    prob.n = n
    prob.sigma_t = rng.uniform(0.5, 4.0, C)
    prob.sigma_s = 0.5 * prob.sigma_t
    prob.q_cell = np.zeros(C)
    prob.inflow = None
    print("case", n, flush=True)
    pr = Pair(prob, with_mg=False)
    lv = pr.op.outer
    g = _rand(lv.A * lv.grid.S, 14)
    ref = lv.sweep(g)
    assert rel(to_np(pr.tr.sweep(0, to_dev(g))), ref) < 1e-12
    assert rel(to_np(pr.tr.sweep(0, to_dev(g), adjoint=True)), lv.sweep_T(g)) < 1e-12
    got32 = pr.tr.sweep(0, to_dev(g).float()).double().cpu().numpy()
    assert rel(got32, ref) < 2e-5
    assert pr.tr.sweep_pair["f32"] == (n[0] % 2 == 0)


def test_coarse_gs_multiblock_planes():
    """A 12^3 grid: planes of up to 127 cells span several workgroups."""
    prob = small(dim=3, n=12, level=0, order=3, seed=15)
    print("case 12^3 level 0", flush=True)
    pr = Pair(prob)
    lv0 = pr.op.mg.levels[0]
    f = _rand(lv0.A * lv0.grid.S, 16)
    assert rel(to_np(pr.tr.coarse_gs(to_dev(f), 2)), pr.op.mg.coarse_gs(f, 2)) < 1e-11
    assert rel(to_np(pr.tr.coarse_gs(to_dev(f), 2, adjoint=True)), pr.op.mg.coarse_gs(f, 2, adjoint=True)) < 1e-11


def test_coarse_gs_bricks_noncubic():
    """An even 6 x 4 x 8 grid: the forward and adjoint solves run over
    2 x 2 x 2 bricks (brick counts differ per axis)."""
    prob = small(dim=3, n=(6, 4, 8), level=0, order=3, seed=17)
    print("case 6x4x8 level 0", flush=True)
    pr = Pair(prob)
    lv0 = pr.op.mg.levels[0]
    f = _rand(lv0.A * lv0.grid.S, 18)
    for nu in (1, 3):
        assert rel(to_np(pr.tr.coarse_gs(to_dev(f), nu)), pr.op.mg.coarse_gs(f, nu)) < 1e-11
        assert rel(to_np(pr.tr.coarse_gs(to_dev(f), nu, adjoint=True)),
                   pr.op.mg.coarse_gs(f, nu, adjoint=True)) < 1e-11


def test_coarse_gs_forms_agree():
    """The dataflow (brick and cell) and barrier forms of the coarse solve
    give the oracle's result; 16 sweeps exceed the dataflow counters' range
    and take the barrier form."""
    import os
    prob = small(dim=3, n=4, level=0, order=3, seed=21)
    print("case 4^3 level 0, forms", flush=True)
    for form in ("", "cell", "barrier", "barrier_fence"):
        os.environ["TR_COARSE_GS"] = form
        try:
            pr = Pair(prob)
        finally:
            os.environ.pop("TR_COARSE_GS", None)
        lv0 = pr.op.mg.levels[0]
        f = _rand(lv0.A * lv0.grid.S, 22)
        for nu in (2, 16):
            ref = pr.op.mg.coarse_gs(f, nu)
            assert rel(to_np(pr.tr.coarse_gs(to_dev(f), nu)), ref) < 1e-11, (form, nu)
            refa = pr.op.mg.coarse_gs(f, nu, adjoint=True)
            assert rel(to_np(pr.tr.coarse_gs(to_dev(f), nu, adjoint=True)), refa) < 1e-11, (form, nu)
        pr.tr.close()
