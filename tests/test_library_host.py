"""Host-side checks of the C-ABI library (no GPU): the shared library loads and
exports every function the header declares; a host-only handle (device -1)
reproduces the oracle's integer decisions exactly and its FV-PLG rows to
rounding; the stored factorizations solve their systems; bad arguments come
back as status codes with a message."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from oracle.discretize import Level
from paper_2410_05865_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cutcell.h")


def _lib():
    from paper_2410_05865_amd import _lib
    try:
        _lib.load()
    except ImportError as e:       # the library is built by __graft_entry__.build()
        pytest.skip(str(e))
    return _lib


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|long long|const char\s*\*)\s*(cc_\w+)\s*\(", text, flags=re.M)))


def test_header_symbols_exported():
    L = _lib()
    names = _declared()
    assert len(names) >= 20, names
    lib = C.CDLL(L.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding wraps exactly the declared calls
    assert sorted(L.EXPORTED) == names


def test_header_enums_match_binding():
    L = _lib()
    text = open(HEADER).read()
    for name in ("CC_OK", "CC_EINVAL", "CC_ENOCONV", "CC_FP64", "CC_MIXED", "CC_LAPLACIAN", "CC_DIRICHLET",
                 "CC_NEUMANN"):
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", text)
        assert m, name
        assert getattr(L, name) == int(m.group(1)), name
    hm = int(re.search(r"#define CC_HISTORY_MAX (\d+)", text).group(1))
    assert L.HISTORY_MAX == hm


CASES = {
    "sphere16": lambda: inputs.sphere_domain(n=16, radius=0.25, n_min=8),
    "ellipsoid32_neumann": lambda: _ell32(),
    "sphere_interior32": lambda: inputs.sphere_interior_problem(32, n_min=16)[0],
    "ellipsoid32_robin": lambda: _ell32(robin=True),
    "ellipsoid32_robin_walls": lambda: _ell32_robin_walls(),
}


def _ell32_robin_walls():
    """Dirichlet ellipsoids, Robin conditions on three walls (FV-PLG rows with
    Robin wall sites)."""
    d = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    d.n_min = 16
    for ob in d.obstacles:
        ob.bc = inputs.DIRICHLET
    R = inputs.ROBIN
    d.wall_bc = (R, 0, R, 0, 0, R)
    d.wall_robin = ((1.0, 0.5), (1.0, 0.0), (2.0, 0.05), (1.0, 0.0), (1.0, 0.0), (0.7, 0.7))
    return d


def _ell32(robin=False):
    d = inputs.ellipsoid_domain(n=32, seed=7, count=2, axes_range=(0.08, 0.14), h_coarse=1 / 16)
    d.wall_bc = (0, 1, 0, 0, 1, 0)
    d.n_min = 16
    if robin:
        # one Robin surface leaning on the value, one leaning on the flux
        for ob, ab in zip(d.obstacles, [(1.0, 0.3), (0.2, 1.0)]):
            ob.bc = inputs.ROBIN
            ob.robin = ab
    return d


@pytest.fixture(scope="module", params=sorted(CASES))
def host_pair(request):
    L = _lib()
    dom = CASES[request.param]()
    P = L.Problem(dom, device=-1)
    sizes = []
    n = dom.n
    while True:
        sizes.append(n)
        if n % 2 or n // 2 < dom.n_min:
            break
        n //= 2
    levels = [Level(dom, s) for s in sizes]
    yield request.param, P, levels
    P.close()


def test_host_build_matches_oracle(host_pair):
    name, P, levels = host_pair
    assert P.num_levels == len(levels)
    for m, lv in enumerate(levels):
        typ, host, vf = P.export_cells(m)
        ot = np.zeros(lv.n ** 3, np.uint8)
        ot[lv.unknowns] = np.where(lv.is_phi1[lv.unknowns], 1, 2)
        assert np.array_equal(typ, ot), (name, m)
        assert np.array_equal(host, lv.host), (name, m)
        cell, cols, vals = P.export_plg(m)
        assert np.array_equal(cell, lv.phi2)
        for r, p in enumerate(lv.phi2):
            oc, ov = lv.plg[lv.uidx[p]]
            assert list(oc) == list(cols[r])
            # min-norm least squares by Householder QR (library) and SVD (oracle)
            assert np.max(np.abs(np.asarray(ov) - vals[r])) <= 1e-11 * np.max(np.abs(ov))
        info = P.level_info(m)
        assert info["n"] == lv.n
        assert info["n_unknowns"] == lv.N
        assert info["n_phi2"] == len(lv.phi2)


def test_factorizations_solve(host_pair):
    name, P, levels = host_pair
    for m in range(P.num_levels):
        assert P.selfcheck_lu(m) < 1e-12, (name, m)
        nd = P.export_lu_nodes(m)
        info = P.level_info(m)
        assert int(nd["p"].sum()) == info["lu_vars"]
        # postorder: every parent comes after its children, heights grow by one or more
        par = nd["parent"]
        for s, q in enumerate(par):
            if q >= 0:
                assert q > s and nd["height"][q] > nd["height"][s]
        # base offsets partition the variables
        order = np.argsort(nd["base"])
        assert np.array_equal(np.cumsum(nd["p"][order])[:-1], nd["base"][order][1:])


def test_errors_are_status_codes():
    L = _lib()
    dom = inputs.sphere_domain(n=16, radius=0.25, n_min=8)
    with pytest.raises(L.CutCellError) as e:
        L.Problem(dom, device=-1, omega=2.5)
    assert e.value.code == L.CC_EINVAL and "omega" in str(e.value)
    with pytest.raises(L.CutCellError) as e:
        L.Problem(dom, device=-1, precision=7)
    assert e.value.code == L.CC_EINVAL
    big = inputs.sphere_domain(n=1292, radius=0.25, n_min=8)     # n^3 beyond 32-bit cell indices
    with pytest.raises(L.CutCellError) as e:
        L.Problem(big, device=-1)
    assert e.value.code == L.CC_EINVAL and "1290" in str(e.value)
    skew = _ell32()
    skew.obstacles[0].rot = skew.obstacles[0].rot * 1.01   # not a rotation
    with pytest.raises(L.CutCellError) as e:
        L.Problem(skew, device=-1)
    assert e.value.code == L.CC_EINVAL and "orthonormal" in str(e.value)
    bad = _ell32(robin=True)
    bad.obstacles[0].robin = (0.0, 0.0)     # no condition at all
    with pytest.raises(L.CutCellError) as e:
        L.Problem(bad, device=-1)
    assert e.value.code == L.CC_EINVAL
    for ab in ((0.0, 0.0), (float("inf"), 1.0)):  # a Robin wall with no condition, or a non-finite one
        badw = _ell32_robin_walls()
        badw.wall_robin = (ab,) + tuple(badw.wall_robin[1:])
        with pytest.raises(L.CutCellError) as e:
            L.Problem(badw, device=-1)
        assert e.value.code == L.CC_EINVAL and "Robin wall" in str(e.value)
    wild = _ell32()
    wild.wall_bc = (0, 1, 0, 0, 7, 0)
    with pytest.raises(L.CutCellError) as e:
        L.Problem(wild, device=-1)
    assert e.value.code == L.CC_EINVAL
    with L.Problem(dom, device=-1) as Q:          # the handle is released on leaving the block
        assert Q.num_levels >= 2
    assert Q._h is None
    P = L.Problem(dom, device=-1)
    with pytest.raises(L.CutCellError) as e:
        P.level_info(5)
    assert e.value.code == L.CC_EINVAL
    lib = L.load()
    info = L.CcSolveInfo()
    rc = lib.cc_solve(P._h, C.c_void_p(16), C.c_void_p(16), C.byref(info))
    assert rc == L.CC_EDEVICE and b"host-only" in lib.cc_last_error()
    P.close()


def test_geometry_plg_and_pivot_failures_are_status_codes():
    """The three failure classes of the set-up, each forced from the host:
    an obstacle in the wall layer and two obstacles in one cell (CC_EGEOM), a
    domain too small for any poised lattice (CC_EPLG; the oracle fails on the
    same domain), and a pivot threshold no pivot can meet (CC_ESINGULAR)."""
    from oracle.discretize import Level, PLGError
    L = _lib()
    with pytest.raises(L.CutCellError) as e:
        L.Problem(inputs.sphere_domain(n=16, radius=0.45, n_min=8), device=-1)
    assert e.value.code == L.CC_EGEOM and "wall layer" in str(e.value)
    two = inputs.sphere_domain(n=16, radius=0.2, n_min=8)
    two.obstacles.append(inputs.Obstacle(np.array([0.5, 0.5, 0.78]), np.full(3, 0.05), np.eye(3), inputs.DIRICHLET))
    with pytest.raises(L.CutCellError) as e:
        L.Problem(two, device=-1)
    assert e.value.code == L.CC_EGEOM and "two obstacles" in str(e.value)
    ball = inputs.Obstacle(np.array([0.5, 0.5, 0.5]), np.full(3, 0.2), np.eye(3), inputs.DIRICHLET)
    tiny = inputs.Domain(n=8, obstacles=[ball], n_min=8, inside=True)    # ~30 cells, fewer than a lattice's 35
    with pytest.raises(L.CutCellError) as e:
        L.Problem(tiny, device=-1)
    assert e.value.code == L.CC_EPLG and "poised lattice" in str(e.value)
    with pytest.raises(PLGError):
        Level(tiny, 8)
    dom = inputs.sphere_domain(n=16, radius=0.25, n_min=8)
    with pytest.raises(L.CutCellError) as e:
        L.Problem(dom, device=-1, pivot_tol=10.0)
    assert e.value.code == L.CC_ESINGULAR and "pivot" in str(e.value)
    for bad in (0.0, -1.0, 1e7, float("nan")):
        with pytest.raises(L.CutCellError) as e:
            L.Problem(dom, device=-1, pivot_tol=bad)
        assert e.value.code == L.CC_EINVAL
    with L.Problem(dom, device=-1, pivot_tol=1e-12) as Q:      # a stricter but attainable threshold
        assert Q.selfcheck_lu(0) < 1e-12


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """No fallback: without the built library every entry point raises."""
    from paper_2410_05865_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libcutcell.so"))
    monkeypatch.setattr(_lib, "_LIB", None)
    with pytest.raises(ImportError):
        _lib.load()
    with pytest.raises(ImportError):
        _lib.Problem(inputs.sphere_domain(n=16, radius=0.25, n_min=8), device=-1)
