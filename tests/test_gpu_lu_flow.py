"""The one-launch LU sweeps (cc_set_lu_schedule with subtree = 2; protocol in
csrc/lu_flow.hpp, proven on the CPU by test_lu_flow_protocol.py) against the
oracle and against the per-height launches of the same factorization: the
LU-correction of every level and the bottom solve, then whole solves with
every level on the one-launch sweeps, eagerly and through the captured graph
replayed several times (the counters are reset by a fill kernel inside the
graph).  A wait that gave up would make the call fail (CC_EDEVICE)."""
import numpy as np
import pytest

from oracle.fields import Field
from oracle.multigrid import Hierarchy, MGParams
from paper_2410_05865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_05865_amd import _lib
    _lib.load()
    return _lib


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


WORK = {"sphere32": lambda: inputs.sphere_domain(n=32, radius=0.25, n_min=16),
        "sphere96_ragged": lambda: inputs.sphere_domain(n=96, radius=0.1, n_min=24)}
_ORACLE = {}


def _oracle(name):
    """(domain, hierarchy) of a workload, built once per module."""
    if name not in _ORACLE:
        dom = WORK[name]()
        _ORACLE[name] = (dom, Hierarchy(dom))
    return _ORACLE[name]


@pytest.mark.parametrize("name", sorted(WORK))
def test_flow_sweeps_match_oracle_and_per_height(name):
    L = _lib()
    dom, H = _oracle(name)
    P = L.Problem(dom, use_graph=0)
    M = len(H.levels) - 1
    rng = np.random.default_rng(8)
    for m in range(M + 1):
        lv, op = H.levels[m], H.ops[m]
        s = rng.standard_normal(lv.N)
        e0 = rng.standard_normal(lv.N) if m < M else None
        ref = op.smo2(e0, s) if m < M else op.lu_all.solve(s)
        sd = _dev(lv.to_grid(s))
        info = P.level_info(m)
        epl = info["lu_entries_per_lane"]
        outs = {}
        for mode in (0, 2):
            print(f"[flow] {name} level {m} mode {mode}", flush=True)
            P.set_lu_schedule(m, epl, mode, 0)
            for rep in range(3):
                ed = _dev(lv.to_grid(e0)) if m < M else _dev(np.zeros(lv.n ** 3))
                if m < M:
                    P.smo2(m, sd, ed)
                else:
                    P.bottom_solve(sd, ed)
                got = ed.cpu().numpy()[lv.unknowns]
                assert _rel(got, ref) < 1e-11, (name, m, mode, rep)
                outs.setdefault(mode, []).append(got)
        # the same factorization either way: only the order of the atomic
        # additions differs
        for got in outs[2]:
            assert _rel(got, outs[0][0]) < 1e-12, (name, m)
    P.close()


@pytest.mark.parametrize("graph", [0, 1])
def test_solves_with_flow_sweeps(graph):
    L = _lib()
    dom, H = _oracle("sphere96_ragged")
    F = Field(inputs.sinprod_field())
    lv = H.fine
    if "solution" not in _ORACLE:
        r0 = H.fine.rhs(F.laplacian_desc(), F)
        _ORACLE["solution"] = (r0,) + tuple(H.solve(r0, MGParams(tol=1e-10)))
    r_or, x_or, hist = _ORACLE["solution"]
    P = L.Problem(dom, use_graph=graph)
    for m in range(P.num_levels):
        P.set_lu_schedule(m, P.level_info(m)["lu_entries_per_lane"], 2, 0)
    r = _dev(lv.to_grid(r_or))
    sols = []
    for rep in range(4):
        print(f"[flow] solve graph {graph} replay {rep}", flush=True)
        phi = _dev(np.zeros(lv.n ** 3))
        info = P.solve(r, phi)
        assert info["converged"] and info["iterations"] == len(hist) - 1
        got = phi.cpu().numpy()[lv.unknowns]
        assert _rel(got, x_or) < 1e-11
        sols.append(got)
    for got in sols[1:]:
        assert _rel(got, sols[0]) < 1e-12
    P.close()
