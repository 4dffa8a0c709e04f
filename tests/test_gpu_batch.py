"""GPU checks of the batched solver: the batched system apply against the
single-configuration apply of every member (same tables, same tree or direct
lists, so they agree to rounding), the lockstep solve against single solves
and against the oracle's stored capture rate of the N=10 workload, graph
replay against kernel-by-kernel launches, and one-patch members."""
import math
from pathlib import Path

import numpy as np
import pytest

import layouts

pytestmark = pytest.mark.gpu
GOLD = Path(__file__).resolve().parent / "golden"
TOL_ID = 1e-12


@pytest.fixture(scope="module")
def torch():
    import torch
    assert torch.cuda.is_available()
    return torch


def _members():
    """(centers, eps, problem): the N=10 workload, plus uneven uniform layouts
    over two more (problem, eps) groups, and a one-patch configuration."""
    c1 = layouts.CONFIGS["cfg1"]
    out = [(layouts.config_layout(c1), c1["eps"], c1["problem"])]
    for k, (N, eps, prob) in enumerate([(60, 0.05, 0), (240, 0.02, 1), (1, 0.05, 0), (130, 0.02, 1),
                                        (25, 0.05, 0), (400, 0.02, 1)]):
        out.append((layouts.uniform_centers(N, eps, 500 + k), eps, prob))
    return out


def _rand(torch, n, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    return torch.from_numpy(g.standard_normal(n) * 0.1).cuda()


@pytest.mark.parametrize("far", ["direct", "tree"])
def test_batch_matvec_matches_members(torch, far):
    import paper_1906_04209_amd as nce
    ff = nce.FAR_DIRECT if far == "direct" else nce.FAR_TREE
    mem = _members()
    if far == "tree":
        mem = [m for m in mem if len(m[0]) >= 25]  # a tree needs a few boxes
    # FP32 at grids 1e-4 and tables 1e-6, the settings of the 2e-5 bound below
    bt = nce.Batch(mem, tol_id=TOL_ID, far_field=ff, tol_grid_fp32=1e-4, tol_id_fp32=1e-6)
    assert bt.ngroups == len({(e, p) for _, e, p in mem})
    assert (bt.far_tree == (1 if far == "tree" else 0)).all()
    x = _rand(torch, bt.n, 11)
    y64 = bt.matvec(x, precision=nce.FP64)
    y32 = bt.matvec(x, precision=nce.MIXED)
    torch.cuda.synchronize()
    for b, (c, eps, prob) in enumerate(mem):
        ctx = nce.Context(c, eps, problem=prob, tol_id=TOL_ID, far_field=ff)
        xb = bt.part(x, b).contiguous()
        ref = ctx.matvec(xb, precision=nce.FP64)
        torch.cuda.synchronize()
        d = (ref - xb).abs().max().item()
        e64 = (bt.part(y64, b) - ref).abs().max().item() / max(d, 1e-300)
        e32 = (bt.part(y32, b) - ref).abs().max().item() / max(d, 1e-300)
        print(f"{far} member {b} N={len(c)} eps={eps} problem={prob}: FP64 {e64:.2e} FP32 {e32:.2e}")
        if len(c) == 1:
            assert (bt.part(y64, b) - xb).abs().max().item() == 0.0
            continue
        assert e64 < 1e-12
        assert e32 < 2e-5
        ctx.close()
    bt.close()


def test_batch_auto_far_choice_and_work(torch):
    import paper_1906_04209_amd as nce
    mem = _members()
    bt = nce.Batch(mem, tol_id=TOL_ID)
    w = bt.work()
    print("far field per member (1 = tree):", bt.far_tree.tolist(), "work", w)
    # the one-patch member has nothing to sum; every member's choice is the
    # cheaper of its tree and its direct lists by operation count
    assert bt.far_tree[3] == 0
    assert w["pairs_near"] > 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_solve_matches_single_and_oracle(torch, precision):
    import paper_1906_04209_amd as nce
    pr = nce.FP64 if precision == "fp64" else nce.MIXED
    mem = _members()
    bt = nce.Batch(mem, tol_id=TOL_ID, tol_gmres=1e-10, precision=pr, max_iter=60)
    r = bt.solve()
    assert r["converged"]
    gold = np.load(GOLD / "cfg1.npz")
    e_or = abs(r["result"][0] - float(gold["capture_rate"])) / float(gold["capture_rate"])
    print(f"{precision}: N=10 capture rate {r['result'][0]:.13f} vs oracle {float(gold['capture_rate']):.13f} "
          f"rel {e_or:.2e}")
    assert e_or < 1e-9
    for b, (c, eps, prob) in enumerate(mem):
        inf = r["info"][b]
        assert inf["rel_residual"] <= 1e-10 * 1.0001
        ctx = nce.Context(c, eps, problem=prob, tol_id=TOL_ID, tol_gmres=1e-10, far_field=nce.FAR_DIRECT)
        s = ctx.solve(want_coeffs=False, want_flux=False)
        ref = s["mu"] if prob == nce.INTERIOR else s["capture_rate"]
        if len(c) == 1:
            # one patch: mu = 1/(3 I . e_0) - 3/5 exactly as the single solve
            assert inf["iters_fp64"] + inf["iters_fp32"] == 0
        rel = abs(r["result"][b] - ref) / abs(ref)
        print(f"  member {b} N={len(c)}: batch {r['result'][b]:.12f} single {ref:.12f} rel {rel:.1e} "
              f"iters fp32 {inf['iters_fp32']} fp64 {inf['iters_fp64']}")
        assert rel < 1e-8
        ctx.close()
    bt.close()


def test_graph_replay_equals_eager(torch):
    import paper_1906_04209_amd as nce
    mem = _members()[:4]
    out = []
    for g in (True, False):
        bt = nce.Batch(mem, tol_id=TOL_ID, precision=nce.MIXED, max_iter=40)
        bt.set_solver(1e-10, 40, nce.MIXED, use_graph=g)
        out.append(bt.solve(want_coeffs=True))
        # a second solve on the same batch replays the captured graph again
        again = bt.solve(want_coeffs=True)
        assert np.array_equal(again["result"], out[-1]["result"])
        bt.close()
    assert np.array_equal(out[0]["result"], out[1]["result"])
    assert torch.equal(out[0]["x"], out[1]["x"])


def test_batch_coarse_and_learned_start(torch):
    """Per-member coarse (and learned) starts give the cold results with fewer
    applies; members with one patch stay exact."""
    import paper_1906_04209_amd as nce
    mem = _members()
    bt = nce.Batch(mem, tol_id=TOL_ID, tol_gmres=1e-10, precision=nce.MIXED, max_iter=60)
    cold = bt.solve()
    bt.set_warm_start(None, True)
    warm = bt.solve()
    assert cold["converged"] and warm["converged"]
    for b in range(len(mem)):
        rel = abs(warm["result"][b] - cold["result"][b]) / abs(cold["result"][b])
        ic, iw = cold["info"][b], warm["info"][b]
        print(f"member {b} N={len(mem[b][0])}: cold {ic['iters_fp32']}+{ic['iters_fp64']} coarse "
              f"{iw['iters_fp32']}+{iw['iters_fp64']} applies, x0 residual {iw['rel_residual_x0']:.2e}, rel {rel:.1e}")
        assert rel < 1e-8
        if len(mem[b][0]) > 1:
            assert iw["rel_residual_x0"] < 0.5 and not iw["used_fallback"]


def test_batch_deflation(torch):
    """The per-member deflation of the mixed inner solves changes how many FP32
    steps a member takes, not what it converges to: the results with and
    without it agree with each other and with deflated single solves; members
    below 64 patches and with one patch are left undeflated; toggling it
    rebuilds the captured step, and a repeated solve is bit-identical."""
    import paper_1906_04209_amd as nce
    spec = [(1500, 0.01, 0), (800, 0.01, 0), (40, 0.01, 0), (1200, 0.02, 1), (1, 0.01, 0), (600, 0.02, 1)]
    mem = [(layouts.uniform_centers(N, eps, 900 + k), eps, prob) for k, (N, eps, prob) in enumerate(spec)]
    bt = nce.Batch(mem, tol_id=1e-10, tol_gmres=1e-10, precision=nce.MIXED, max_iter=60)
    on = bt.solve()
    bt.set_deflation(False)
    off = bt.solve()
    bt.set_deflation(True)
    again = bt.solve()
    assert on["converged"] and off["converged"] and again["converged"]
    assert np.array_equal(again["result"], on["result"])
    n_on = n_off = 0
    for b, (c, eps, prob) in enumerate(mem):
        i_on, i_off = on["info"][b], off["info"][b]
        rel = abs(on["result"][b] - off["result"][b]) / abs(off["result"][b])
        ctx = nce.Context(c, eps, problem=prob, tol_id=1e-10, tol_gmres=1e-10, precision=nce.MIXED)
        s = ctx.solve(want_coeffs=False, want_flux=False)
        ref = s["mu"] if prob == nce.INTERIOR else s["capture_rate"]
        rel_single = abs(on["result"][b] - ref) / abs(ref)
        print(f"member {b} N={len(c)}: FP32 steps deflated {i_on['iters_fp32']} plain {i_off['iters_fp32']}; "
              f"on vs off {rel:.1e}, vs single deflated solve {rel_single:.1e} (single {s['iters_fp32']} steps)")
        assert i_on["rel_residual"] <= 1e-10 * 1.0001 and i_off["rel_residual"] <= 1e-10 * 1.0001
        assert rel < 1e-8 and rel_single < 1e-8
        if len(c) < 64:
            assert i_on["iters_fp32"] == i_off["iters_fp32"]
        else:
            n_on += i_on["iters_fp32"]
            n_off += i_off["iters_fp32"]
        ctx.close()
    assert n_on < n_off
    bt.close()
