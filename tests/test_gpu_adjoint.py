"""GPU parity of the hand-written adjoint (sabr_cost_vjp) and of the
Levenberg-Marquardt polish (sabr_lm_polish) against the CPU oracle's
dual-number gradient and LM, central finite differences and gradcheck."""
import numpy as np
import pytest

from conftest import complete_with_oracle
from paper_2408_01470_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_01470_amd import api as A
    return A


def _points(model, truth, n, seed):
    lb, ub = I.box(model)
    g = np.random.default_rng(seed)
    near = np.clip(truth[None, :] * g.uniform(0.85, 1.15, (n, len(lb))), lb, ub)
    return np.vstack([truth[None, :], near])


def _grad_close(g_gpu, g_ora, rtol, what):
    scale = np.maximum(np.abs(g_ora), 1e-6 * np.abs(g_ora).max(axis=1, keepdims=True))
    err = np.abs(g_gpu - g_ora) / scale
    i, k = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= rtol, (f"{what}: gradient rel err {err.max():.3e} at point {i} "
                               f"param {k}: gpu {g_gpu[i, k]!r} oracle {g_ora[i, k]!r}")


MARKETS = [
    ("caplets-vol", dict(kind="caplet", formula=0, residual=0)),
    ("caplets-price", dict(kind="caplet", formula=0, residual=1)),
    ("caplets-eq3", dict(kind="caplet", formula=1, residual=0)),
    ("caplets-eq3-price", dict(kind="caplet", formula=1, residual=1)),
    ("lmm-price", dict(kind="lmm", formula=0, residual=1)),
    ("lmm-vol-eq3", dict(kind="lmm", formula=1, residual=0)),
]


def _market(oracle, spec):
    if spec["kind"] == "caplet":
        m, truth, noise = I.caplet_market(formula=spec["formula"], residual=spec["residual"])
    else:
        m, truth, noise = I.lmm_market(M=14, n_cap_K=7, n_exp=6, n_ten=7, n_swp_K=5,
                                       residual=spec["residual"])
        m = dict(m, formula=spec["formula"])
    return complete_with_oracle(oracle, m, truth, noise), truth


@pytest.mark.parametrize("name,spec", MARKETS, ids=[m[0] for m in MARKETS])
def test_vjp_matches_oracle_dual_gradient(api, oracle, name, spec):
    mk, truth = _market(oracle, spec)
    plan = api.Plan(mk)
    model = mk["model"]
    pts = _points(model, truth[0], 24, 5)
    c_o, g_o, A_o, b_o = oracle.cost_grad(mk, pts, normal=True)
    out = plan.vjp(torch.tensor(pts, device="cuda"), normal=True)
    c_g = out["cost"].cpu().numpy()
    fin = np.isfinite(c_o)
    assert fin.sum() >= 10
    assert np.array_equal(fin, np.isfinite(c_g))
    np.testing.assert_allclose(c_g[fin], c_o[fin], rtol=1e-12)
    _grad_close(out["grad"].cpu().numpy()[fin], g_o[fin], 1e-10, name)
    A_g = out["jtwj"].cpu().numpy()[fin]
    sA = np.abs(A_o[fin]).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(A_g - A_o[fin]) / sA) <= 1e-10, name
    _grad_close(out["jtwr"].cpu().numpy()[fin], b_o[fin], 1e-10, name + " J^T W r")
    # outside the domain: +inf cost and zero gradient
    g_bad = plan.vjp(torch.tensor(pts[~fin], device="cuda"))["grad"].cpu().numpy() \
        if (~fin).any() else np.zeros((0, len(pts[0])))
    assert np.all(g_bad == 0.0)


def test_vjp_against_central_differences_1000_points(api, oracle, c1_market):
    """Config 4's check: 1000 random points, central differences with an
    absolute step h = 1e-6 per coordinate on the GPU cost."""
    mk, truth = c1_market
    plan = api.Plan(mk)
    lb, ub = I.box(0)
    h = 1e-6
    pts = I.random_box_points(0, 1000, 77)
    pts = np.clip(pts, lb + 2 * h, ub - 2 * h)
    P = len(lb)
    grad = plan.vjp(torch.tensor(pts, device="cuda"))["grad"].cpu().numpy()
    pm = np.concatenate([pts + h * np.eye(P)[k] for k in range(P)] +
                        [pts - h * np.eye(P)[k] for k in range(P)])
    c = plan.cost(torch.tensor(pm, device="cuda")).cpu().numpy().reshape(2 * P, len(pts))
    fd = ((c[:P] - c[P:]) / (2 * h)).T
    ok = np.all(np.isfinite(fd), axis=1) & np.all(np.isfinite(grad), axis=1)
    assert ok.sum() > 900
    scale = np.maximum(np.abs(fd[ok]), 1e-3 * np.abs(fd[ok]).max(axis=1, keepdims=True))
    err = np.abs(grad[ok] - fd[ok]) / scale
    assert np.quantile(err, 0.999) <= 1e-6, f"worst {err.max():.2e}"


def test_autograd_function_gradcheck(api, oracle, c1_market):
    mk, truth = c1_market
    plan = api.Plan(mk)
    x = torch.tensor(_points(0, truth[0], 3, 9), device="cuda", requires_grad=True)
    f = lambda p: api.sabr_cost(plan, p)
    assert torch.autograd.gradcheck(f, (x,), eps=1e-7, atol=1e-7, rtol=1e-5)
    y = api.sabr_cost(plan, x).sum()
    y.backward()
    _, g_o = oracle.cost_grad(mk, x.detach().cpu().numpy())
    _grad_close(x.grad.cpu().numpy(), g_o, 1e-10, "autograd")


@pytest.mark.parametrize("which", ["caplets", "lmm"])
def test_lm_polish_matches_oracle(api, oracle, c1_market, c2_market, which):
    mk, truth = c1_market if which == "caplets" else c2_market
    model = mk["model"]
    lb, ub = I.box(model)
    g = np.random.default_rng(3)
    starts = np.clip(truth[0][None, :] * g.uniform(0.9, 1.1, (6, len(lb))), lb, ub)
    if which == "caplets":
        starts[0, 1] = 1.0                 # on the beta bound
        lb2, ub2 = lb.copy(), ub.copy()
    else:
        lb2, ub2 = lb.copy(), ub.copy()
        lb2[10] = ub2[10] = starts[0, 10]  # eta2 fixed: a frozen coordinate
        starts[:, 10] = starts[0, 10]
    plan = api.Plan(mk)
    xg, fg, itg = plan.lm(torch.tensor(starts, device="cuda"), lb2, ub2, max_iter=25)
    xo, fo, ito = oracle.lm_polish(mk, starts, None, lb2, ub2, max_iter=25)
    fg = fg.cpu().numpy()
    np.testing.assert_allclose(fg, fo, rtol=1e-8)
    f0 = oracle.cost_batch(mk, starts)
    assert np.all(fg <= f0)
    xg = xg.cpu().numpy()
    assert np.all(xg >= lb2) and np.all(xg <= ub2)
    assert np.all(xg[:, 10] == lb2[10]) if which == "lmm" else True


def test_vjp_full_size_long_swaps(api, oracle):
    """The 64-market workload at full size (8838 quotes, swaps of up to 20
    forwards): gradient, J^T W J and J^T W r of sampled points of three
    markets against the oracle's dual numbers."""
    from paper_2408_01470_amd import workloads as W
    w = W.config5()

    def vols(vm, truth):
        M = oracle.Market(vm)
        out = []
        for i in range(M.n_inst):
            mv, _, _, ok = oracle.model_values(M, i, truth[i])
            assert ok
            out.append(mv)
        return np.concatenate(out)

    mk = W.synthesize(w, vols)
    assert max(mk["und_len"]) == 20
    g = np.random.default_rng(8)
    insts = np.array([0, 0, 31, 63, 63], np.int32)
    lb, ub = I.box(1)
    pts = np.clip(w.truth[insts] * g.uniform(0.93, 1.07, (len(insts), 12)), lb, ub)
    c_o, g_o, A_o, b_o = oracle.cost_grad(mk, pts, insts, normal=True)
    plan = api.Plan(mk)
    out = plan.vjp(torch.tensor(pts, device="cuda"), pt_inst=torch.tensor(insts, device="cuda"),
                   normal=True)
    np.testing.assert_allclose(out["cost"].cpu().numpy(), c_o, rtol=1e-12)
    _grad_close(out["grad"].cpu().numpy(), g_o, 1e-10, "c5")
    A_g = out["jtwj"].cpu().numpy()
    sA = np.abs(A_o).max(axis=(1, 2), keepdims=True)
    assert np.max(np.abs(A_g - A_o) / sA) <= 1e-10
    _grad_close(out["jtwr"].cpu().numpy(), b_o, 1e-10, "c5 J^T W r")


GRAD_MARKETS = [
    ("lmm-price", dict(M=14, n_cap_K=7, n_exp=6, n_ten=7, n_swp_K=5, formula=0, residual=1)),
    ("lmm-vol", dict(M=14, n_cap_K=7, n_exp=6, n_ten=7, n_swp_K=5, formula=0, residual=0)),
    ("lmm-vol-eq3", dict(M=14, n_cap_K=7, n_exp=6, n_ten=7, n_swp_K=5, formula=1, residual=0)),
    ("lmm-price-eq3", dict(M=14, n_cap_K=7, n_exp=6, n_ten=7, n_swp_K=5, formula=1, residual=1)),
    # swaps of 17..24 forwards (register columns of 24) and beyond 24 (LDS columns)
    ("lmm-price-len22", dict(M=26, n_cap_K=3, n_exp=4, n_ten=22, n_swp_K=3, formula=0,
                             residual=1)),
    ("lmm-price-len30", dict(M=34, n_cap_K=3, n_exp=3, n_ten=30, n_swp_K=3, formula=0,
                             residual=1)),
]


@pytest.mark.parametrize("name,spec", GRAD_MARKETS, ids=[m[0] for m in GRAD_MARKETS])
def test_gradient_without_normal_equations(api, oracle, name, spec):
    """sabr_cost_vjp without J^T W J (the per-underlying seeds and one map
    sweep each) against the oracle's dual-number gradient, and against the
    same call with J^T W J (the map-Jacobian path); ragged multi-market
    batches with interleaved instances, an invalid instance index and
    out-of-domain points."""
    sp = dict(spec)
    formula, residual = sp.pop("formula"), sp.pop("residual")
    m, truth, noise = I.lmm_market(n_markets=3, residual=residual, seed=I.SEED_BASE + 4100, **sp)
    m = dict(m, formula=formula)
    mk = complete_with_oracle(oracle, m, truth, noise)
    plan = api.Plan(mk)
    g = np.random.default_rng(11)
    insts = np.array([0, 2, 1, 0, 2, 2, 1, 0, 1, 2, 0, 0, 1], np.int32)
    lb, ub = I.box(1)
    pts = np.clip(truth[insts] * g.uniform(0.85, 1.15, (len(insts), 12)), lb, ub)
    pts[3, 8] = 0.999999                   # |rho| < 1 still
    pts[5, 10] = 1.0                       # eta2 on its bound
    bad = pts[7].copy()
    bad[0], bad[3] = -0.05, 0.0            # alpha(T) < 0 for every forward: out of domain
    pts = np.vstack([pts, bad])
    insts = np.append(insts, 1).astype(np.int32)
    c_o, g_o = oracle.cost_grad(mk, pts, insts)
    fin = np.isfinite(c_o)
    assert fin.sum() >= 10 and not fin[-1]
    P = torch.tensor(pts, device="cuda")
    pi = torch.tensor(insts, device="cuda")
    gc = torch.tensor(g.uniform(0.5, 2.0, len(pts)), device="cuda")
    out = plan.vjp(P, pt_inst=pi, want_jtwr=True)
    c_g = out["cost"].cpu().numpy()
    assert np.array_equal(fin, np.isfinite(c_g))
    # the same per-quote arithmetic as the cost kernel (summation order aside)
    c_k = plan.cost(P, pt_inst=pi).cpu().numpy()
    np.testing.assert_allclose(c_g[fin], c_k[fin], rtol=1e-14)
    # Against the oracle: 1e-12, except for swaps beyond 24 forwards in price
    # mode.  There the map's O(n) recursions and the oracle's O(n^2) pair sums
    # round apart by about n ulps in (alpha_S, rho_S, nu_S), and the deep
    # out-of-the-money Black prices of the 0.8 log-moneyness strikes (down to
    # 1e-35) amplify a relative vol difference by d ln m/d ln sigma = vega
    # sigma/m, about d1^2 ~ 100: measured 1.1e-12 on the cost, while the vols
    # themselves agree to 1e-12 (checked below in vol mode).
    long_price = residual == I.RESID_PRICE and max(mk["und_len"]) > 24
    np.testing.assert_allclose(c_g[fin], c_o[fin], rtol=5e-12 if long_price else 1e-12)
    if residual == I.RESID_PRICE:
        vm = I.as_vol_market(mk)
        _, mv = api.Plan(vm).cost(P, pt_inst=pi, model=True)
        mv = mv.cpu().numpy()
        nq = np.diff(mk["q_off"])
        for i in np.nonzero(fin)[0]:
            mo, _, _, ok = oracle.model_values(vm, int(insts[i]), pts[i])
            assert ok
            q = nq[insts[i]]
            assert np.max(np.abs(mv[i, :q] - mo) / mo) <= 1e-12, f"point {i}: vols"
    g_g = out["grad"].cpu().numpy()
    _grad_close(g_g[fin], g_o[fin], 1e-10, name)
    assert np.all(g_g[~fin] == 0.0)
    # J^T W r is half the gradient; g_cost scales it
    ref = plan.vjp(P, pt_inst=pi, normal=True)
    _grad_close(out["jtwr"].cpu().numpy()[fin], ref["jtwr"].cpu().numpy()[fin], 1e-10,
                name + " J^T W r")
    scaled = plan.vjp(P, pt_inst=pi, g_cost=gc)["grad"].cpu().numpy()
    np.testing.assert_allclose(scaled[fin], g_g[fin] * gc.cpu().numpy()[fin, None], rtol=1e-15)
    # an instance index out of range: NaN cost, zero gradient
    o2 = plan.vjp(P[:2], pt_inst=torch.tensor([0, 7], dtype=torch.int32, device="cuda"))
    assert np.isnan(o2["cost"][1].item()) and np.isfinite(o2["cost"][0].item())


def test_gradient_without_normal_equations_full_size(api, oracle):
    """The 64-market workload at full size (8838 quotes, swaps of up to 20
    forwards), interleaved instances: gradient against the oracle."""
    from paper_2408_01470_amd import workloads as W
    w = W.config5()

    def vols(vm, truth):
        M = oracle.Market(vm)
        out = []
        for i in range(M.n_inst):
            mv, _, _, ok = oracle.model_values(M, i, truth[i])
            assert ok
            out.append(mv)
        return np.concatenate(out)

    mk = W.synthesize(w, vols)
    g = np.random.default_rng(18)
    insts = np.array([0, 31, 0, 63, 63, 31, 5, 0, 63], np.int32)
    lb, ub = I.box(1)
    pts = np.clip(w.truth[insts] * g.uniform(0.93, 1.07, (len(insts), 12)), lb, ub)
    c_o, g_o = oracle.cost_grad(mk, pts, insts)
    plan = api.Plan(mk)
    out = plan.vjp(torch.tensor(pts, device="cuda"), pt_inst=torch.tensor(insts, device="cuda"))
    np.testing.assert_allclose(out["cost"].cpu().numpy(), c_o, rtol=1e-12)
    _grad_close(out["grad"].cpu().numpy(), g_o, 1e-10, "c5 gradient")
