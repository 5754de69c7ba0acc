"""Every device sweep schedule of the LU-correction and the bottom solve
(factor entries per lane, wavefront cap, subtree launch), set through the C ABI,
against the oracle on the small parity workloads; the subtree launches, which
only larger factorizations have, against the oracle-checked per-height
schedule of the same problem."""
import numpy as np
import pytest

from oracle.multigrid import Hierarchy
from paper_2410_05865_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EPL = (2, 4, 8, 16, 32)
CAPS = (0, 4, 64)   # none; 4 wavefronts (long task loops, lone last tasks); 64


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


def _workloads():
    ell = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    ell.wall_bc = (0, 1, 0, 0, 1, 0)
    ell.n_min = 16
    return {"sphere32": inputs.sphere_domain(n=32, radius=0.25, n_min=16),
            "ellipsoid32_neumann": ell,
            "sphere96_ragged": inputs.sphere_domain(n=96, radius=0.1, n_min=24)}


WORK = _workloads()


@pytest.mark.parametrize("name", sorted(WORK))
def test_every_schedule_matches_oracle(name):
    L = _lib()
    dom = WORK[name]
    H = Hierarchy(dom)
    P = L.Problem(dom, use_graph=0)
    M = len(H.levels) - 1
    rng = np.random.default_rng(5)
    for m in range(M + 1):
        lv, op = H.levels[m], H.ops[m]
        s = rng.standard_normal(lv.N)
        if m < M:
            e0 = rng.standard_normal(lv.N)
            ref = op.smo2(e0, s)
        else:
            ref = op.lu_all.solve(s)
        sd = _dev(lv.to_grid(s))
        info = P.level_info(m)
        print(f"[schedules] {name} level {m}: chosen {info['lu_entries_per_lane']} entries per lane, "
              f"cap {info['lu_waves_cap']}, subtrees {info['lu_subtrees']}", flush=True)
        for epl in EPL:
            for cap in CAPS:
                P.set_lu_schedule(m, epl, 0, cap)
                if m < M:
                    ed = _dev(lv.to_grid(e0))
                    P.smo2(m, sd, ed)
                else:
                    ed = _dev(np.zeros(lv.n ** 3))
                    P.bottom_solve(sd, ed)
                err = _rel(ed.cpu().numpy()[lv.unknowns], ref)
                assert err < 1e-11, (name, m, epl, cap, err)
    P.close()


def test_subtree_schedules_agree():
    """128^3 ellipsoid workload: its level-0 factorization has a subtree launch.
    Every subtree schedule reproduces the per-height schedule's LU-correction to
    rounding (the per-height kernels are the ones checked against the oracle
    above, at every entries-per-lane value)."""
    L = _lib()
    dom, _ = inputs.ellipsoid_workload(128, seed=1)
    P = L.Problem(dom, use_graph=0)
    trials = P.level_info(0)["lu_tune_ms"]
    assert trials[1] > 0          # the build-time trial ran a subtree launch
    P.set_lu_schedule(0, 2, 1, 0)
    info = P.level_info(0)
    print(f"[schedules] ellipsoid128 level 0: {info['lu_subtrees']} subtrees below height "
          f"{info['lu_subtree_cut']}, trials {[round(v, 4) for v in trials]}", flush=True)
    assert info["lu_subtrees"] > 0
    n3 = 128 ** 3
    g = torch.Generator(device="cpu").manual_seed(9)
    s = torch.randn(n3, generator=g, dtype=torch.float64).cuda()
    e0 = torch.randn(n3, generator=g, dtype=torch.float64).cuda()
    P.set_lu_schedule(0, 4, 0, 0)
    ref = e0.clone()
    P.smo2(0, s, ref)
    for epl in EPL:
        for cap in (0, 4):
            P.set_lu_schedule(0, epl, 1, cap)
            ed = e0.clone()
            P.smo2(0, s, ed)
            err = float((ed - ref).abs().max() / ref.abs().max())
            assert err < 1e-12, (epl, cap, err)
    with pytest.raises(L.CutCellError):
        P.set_lu_schedule(0, 3, 0, 0)
    P.close()
