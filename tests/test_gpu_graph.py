"""Graph replay (eik_opts.graph): a repeated problem set replays its captured
launch sequence.  Every replay is checked against the eager solve, with the
program's own eager work and synchronisations between replays; buffer
contents may change between replays; a workspace that grows drops its graphs."""
import numpy as np
import pytest

import oracle as O
from paper_1110_6220_amd import workloads as W
from gpu_util import f32_bound, max_abs, max_rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eik():
    import torch
    assert torch.cuda.is_available()
    from paper_1110_6220_amd import eik as E
    return E


def host(u):
    return u.double().cpu().numpy()


def test_single_problem_replays_match_eager(eik):
    import torch
    w = W.random_small(np.random.default_rng(70), 300, 257, obst=0.1, nsrc=3, q_spread=0.1)
    d = to_dev(w)
    U = O.fmm(O.Problem.from_workload(w))
    print("[gpu] graph replay: single problem", flush=True)
    eager, _ = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d["mask"])
    eager = host(eager)
    assert max_rel(eager, U) <= 1e-12
    u = torch.empty_like(d["F"])
    other = to_dev(W.smooth_sine(129, 0.3))
    replays = 0
    for rep in range(4):
        u.fill_(-1.0)
        _, st = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], d["mask"], u_out=u, graph=True)
        torch.cuda.synchronize()
        got = host(u)
        assert max_rel(got, eager) <= 1e-12, rep
        assert max_rel(got, U) <= 1e-12, rep
        replays += st["graph_replayed"]
        # the program's own eager work between replays
        eik.eik_solve(other["F"], other["h"], other["src"], other["q"])
        torch.cuda.synchronize()
    assert replays >= 2


def test_changed_contents_replay(eik):
    import torch
    w = W.smooth_sine(257, 0.5)
    d = to_dev(w)
    u = torch.empty_like(d["F"])
    print("[gpu] graph replay: changed speeds", flush=True)
    eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u, graph=True)
    for amp in (0.2, 0.7):
        w2 = W.smooth_sine(257, amp)
        d["F"].copy_(torch.from_numpy(w2["F"]))  # same buffer, new contents
        _, st = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u, graph=True)
        assert st["graph_replayed"] == 1
        assert max_rel(host(u), O.fmm(O.Problem.from_workload(w2))) <= 1e-12, amp


CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_1110_6220_amd import eik, workloads as W
dev = torch.device("cuda:0")
def put(w):
    return dict(F=torch.from_numpy(w["F"]).to(dev), src=torch.from_numpy(w["src"]).to(dev),
                q=torch.from_numpy(w["q"]).to(dev), h=w["h"])
a, big = put(W.smooth_sine(257, 0.5)), put(W.smooth_sine(2049, 0.5))
u = torch.empty_like(a["F"])
flags = []
for _ in range(2):
    _, st = eik.eik_solve(a["F"], a["h"], a["src"], a["q"], None, u_out=u, graph=True)
    flags.append(st["graph_replayed"])
eik.eik_solve(big["F"], big["h"], big["src"], big["q"], None)  # grows the workspace
u.fill_(-1.0)
_, st = eik.eik_solve(a["F"], a["h"], a["src"], a["q"], None, u_out=u, graph=True)
flags.append(st["graph_replayed"])
_, st = eik.eik_solve(a["F"], a["h"], a["src"], a["q"], None, u_out=u, graph=True)
flags.append(st["graph_replayed"])
np.save(sys.argv[2], u.cpu().numpy())
print(json.dumps(flags))
"""


def test_workspace_growth_drops_graphs(tmp_path):
    """In a fresh process: a captured graph is replayed, a larger problem
    grows the workspace (its buffers move), the graph is dropped and captured
    again, and the results stay exact."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = tmp_path / "u.npy"
    print("[gpu] graph replay: workspace growth (child process)", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD, root, str(out)], capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    flags = json.loads(r.stdout.strip().splitlines()[-1])
    assert flags == [0, 1, 0, 1], flags
    U = O.fmm(O.Problem.from_workload(W.smooth_sine(257, 0.5)))
    assert max_rel(np.load(out), U) <= 1e-12


def test_batch_replays_match_eager(eik):
    import torch
    ws = W.batch_bumps(count=12, seed=71, n_lo=40, n_hi=300)
    ds = [to_dev(w) for w in ws]
    refs = [O.fmm(O.Problem.from_workload(w)) for w in ws]
    outs = [torch.empty_like(d["F"]) for d in ds]
    for d, u in zip(ds, outs):
        d["u_out"] = u
    print("[gpu] graph replay: batch", flush=True)
    replays = 0
    for rep in range(3):
        for u in outs:
            u.fill_(-1.0)
        _, st = eik.eik_solve_batched(ds, graph=True)
        torch.cuda.synchronize()
        for w, u, U in zip(ws, outs, refs):
            assert max_rel(host(u), U) <= 1e-12, (rep, w["name"])
        replays += st[0]["graph_replayed"]
        x = torch.randn(1 << 20, device="cuda:0")
        (x * 2).sum().item()  # unrelated eager work and a synchronisation
    assert replays == 2


def test_fp32_residual_check_replays(eik):
    import torch
    w = W.config(2)
    d = to_dev(w, "f32")
    U = O.fmm(O.Problem.from_workload(w))
    b = f32_bound(w, U)
    u = torch.empty_like(d["F"])
    print("[gpu] graph replay: FP32 with residual check", flush=True)
    for rep in range(3):
        _, st = eik.eik_solve(d["F"], d["h"], d["src"], d["q"], None, u_out=u, dtype="f32",
                              residual_check=True, graph=True)
        assert max_abs(host(u), U) <= b, rep
        assert 0.0 <= st["max_residual"] <= 4 * 2.0 ** -24 or st["fell_back_to_f64"]
        assert st["graph_replayed"] == (1 if rep else 0)
