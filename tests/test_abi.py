"""The C-ABI library loads and exports every entry point declared in include/nbgs.h (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            names += re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(nbgs_[a-z_0-9]+)\s*\(", txt, re.M)
    return sorted(set(names))


def test_header_declares_entry_points():
    names = _declared()
    for want in ("nbgs_scene_create", "nbgs_detect", "nbgs_solve", "nbgs_integrate", "nbgs_step"):
        assert want in names


def test_library_exports_every_declared_symbol():
    import paper_1501_05810_amd as nb

    L = ctypes.CDLL(nb.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    # the binding wraps exactly the declared set
    assert sorted(n for n, _, _ in nb._SIGNATURES) == _declared()
    assert nb.nbgs_abi_version() == 2


def test_binding_has_no_cpu_fallback(tmp_path, monkeypatch):
    import paper_1501_05810_amd as nb

    monkeypatch.setattr(nb, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(nb, "_lib", None)
    with pytest.raises(ImportError):
        nb.lib()


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_1501_05810_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt and "nbgs_ref" not in txt, f


def _dummy_bodies(nb, n):
    # argument validation rejects these calls before any device pointer is touched
    return nb.nbgs_bodies(n=n, **{f: 0x1000 for f in nb.BODY_FIELDS})


def _domains_params(nb, k, dts=None, warm=None):
    import ctypes as C

    doms = (nb.nbgs_domain * k)()
    pars = (nb.nbgs_params * k)()
    for i in range(k):
        doms[i] = nb.nbgs_domain(lo=(C.c_double * 3)(0, 0, 0), hi=(C.c_double * 3)(1, 1, 1),
                                 periodic=(C.c_int32 * 3)(0, 0, 0), n_planes=0, planes=None)
        pars[i] = nb.nbgs_params(dt=(dts[i] if dts else 1e-3), gravity=(C.c_double * 3)(0, 0, -9.81), mu=0.3 + 0.1 * i,
                                 tau=0.005, relax=1.0, erp=1.0, precision=0,
                                 warm_start=warm if warm is not None else 1, colour_seed=i)
    return doms, pars


@pytest.mark.parametrize("case", ["dt differs", "learned", "offsets", "empty scene", "no scenes"])
def test_batch_create_rejects_bad_arguments(case):
    """Host-side validation of nbgs_batch_create (the status and message, no device work)."""
    import ctypes as C

    import paper_1501_05810_amd as nb

    L = nb.lib()
    k = 3
    offs = [0, 4, 9, 12]
    dts = [1e-3, 1e-3, 2e-3] if case == "dt differs" else None
    doms, pars = _domains_params(nb, k, dts, warm=2 if case == "learned" else None)
    if case == "offsets":
        offs = [0, 4, 9, 11]
    if case == "empty scene":
        offs = [0, 4, 4, 12]
    n = 0 if case == "no scenes" else k
    arr = (C.c_int64 * 4)(*offs)
    out = C.c_void_p()
    st = L.nbgs_batch_create(n, arr, C.byref(_dummy_bodies(nb, 12)), doms, pars, None, None, 0, None,
                             C.byref(out))
    want = 8 if case == "learned" else 1  # UNSUPPORTED, INVALID_ARG
    assert st == want, (case, st, nb.nbgs_last_error())
    assert not out.value
    msg = nb.nbgs_last_error()
    assert msg


def test_tuning_rejects_unsupported_shapes():
    """nbgs_set_tuning validates before touching the scene: a NULL scene is INVALID_ARG."""
    import ctypes as C

    import paper_1501_05810_amd as nb

    t = nb.nbgs_tuning(block=96, contacts_per_thread=1, xcd_remap=1, nontemporal=0, full_store=0, persistent=0,
                       graph=0)
    assert nb.lib().nbgs_set_tuning(None, 0, C.byref(t)) == 1


def test_workspace_queries_are_host_only_and_grow_with_the_workload():
    """The workspace sizes are pure host computations (no device needed): linear in bodies and contacts, one cell
    table more per batched scene, and the network's in the samples its store holds."""
    import paper_1501_05810_amd as nb

    q = nb.nbgs_workspace_query
    base = q(1000, 0)
    assert base > 16 << 20
    assert base % 256 == 0 and q(12345, 6789) % 256 == 0  # whole aligned blocks
    assert q(2000, 0) - base == pytest.approx(1.1 * 567 * 1000, abs=256)
    assert q(1000, 5000) - base == pytest.approx(1.1 * 1000 * 5000, abs=256)
    assert nb.nbgs_batch_workspace_query(3, 1000, 0) - base == pytest.approx(1.1 * 2 * (65536 * 11.25 + 4096), abs=256)
    m0, m1 = nb.nbgs_mlp_workspace_query(0), nb.nbgs_mlp_workspace_query(1 << 20)
    assert m1 - m0 == pytest.approx(1.1 * 64 * (1 << 20), abs=256)
    with pytest.raises(nb.NbgsError):
        q(-1, 0)


def test_scene_create_needs_a_workspace():
    """Without a workspace (NULL, or smaller than one aligned block) the scene is refused before any device work:
    the library allocates no device memory of its own."""
    import ctypes as C

    import paper_1501_05810_amd as nb

    doms, pars = _domains_params(nb, 1)
    out = C.c_void_p()
    L = nb.lib()
    for ws, size in ((None, 0), (None, 1 << 20), (0x100000, 100)):
        st = L.nbgs_scene_create(C.byref(_dummy_bodies(nb, 12)), C.byref(doms[0]), C.byref(pars[0]), ws, size,
                                 None, C.byref(out))
        assert st == 1 and not out.value and "workspace" in nb.nbgs_last_error()


def test_no_device_allocation_in_the_library_sources():
    """Every device buffer is carved from the caller's workspace: no allocation call in the library's sources."""
    pkg = os.path.join(ROOT, "paper_1501_05810_amd", "csrc")
    pat = re.compile(r"\bhip(Malloc|MallocAsync|MallocManaged|ExtMallocWithFlags|MallocPitch|Malloc3D|Free|FreeAsync)\s*\(")
    for f in sorted(os.listdir(pkg)):
        txt = open(os.path.join(pkg, f)).read()
        assert not pat.search(txt), f
