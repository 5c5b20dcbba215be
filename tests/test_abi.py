"""CPU checks of the C boundary: the library loads and exports every symbol
the public header declares; host-side argument validation (no GPU work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "parapn.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(parapn_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["parapn_create", "parapn_destroy", "parapn_solve", "parapn_pararts", "parapn_workspace_size",
              "parapn_filter_combine", "parapn_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2310_01145_amd as pp

    lib = pp.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(pp.EXPORTED) == declared_functions()


def test_workspace_size_and_validation_on_host():
    import paper_2310_01145_amd as pp

    pb = pp.make_problem("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 12, precision="fp32")
    n32 = pp.workspace_size(pb)
    pb64 = pp.make_problem("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 12, precision="fp64")
    n64 = pp.workspace_size(pb64)
    assert 1.9 * n32 < n64 < 2.1 * n32
    # footprint grows linearly in N
    pb2 = pp.make_problem("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 13, precision="fp32")
    assert 1.9 * n32 < pp.workspace_size(pb2) < 2.1 * n32
    # the coarse-grid start adds its scratch (nodes, gains, bridge weights)
    pbc = pp.make_problem("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 12, precision="fp32",
                          init="coarse")
    assert pp.workspace_size(pbc) > n32
    # the method-of-lines chain under DiagonalEK1 runs as d decoupled problems
    # of state size q+1: its workspace grows linearly in d (the dense EK1
    # engine's with d^2), and the objective rule is accepted there
    mk = lambda d, lin: pp.make_problem("mol_heat_reaction", [0.01], [0.5] * d, 0.0, 1.0, 2, 1024,
                                        precision="fp32", linearization=lin)
    w16, w32 = pp.workspace_size(mk(16, "diag_ek1")), pp.workspace_size(mk(32, "diag_ek1"))
    assert 1.8 * w16 < w32 < 2.2 * w16
    assert pp.workspace_size(mk(32, "ek1")) > 10 * w32
    pp.workspace_size(pp.make_problem("mol_heat_reaction", [0.01], [0.5] * 8, 0.0, 1.0, 2, 10,
                                      linearization="ek0", stop_rule="objective"))
    bad = [
        pp.make_problem("fhn", [0.2, 0.2], [-1.0, 1.0], 0.0, 1.0, 3, 100),         # too few params
        pp.make_problem("fhn", [0.2, 0.2, 3.0], [-1.0], 0.0, 1.0, 3, 100),          # d mismatch
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 5, 100),                   # q out of range
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 0),                     # N < 1
        pp.make_problem("logistic", [], [0.1], 1.0, 1.0, 2, 10),                    # empty span
        pp.make_problem(42, [], [0.1], 0.0, 1.0, 2, 10, d=1),                       # unknown field
        pp.make_problem("logistic", [], [float("nan")], 0.0, 1.0, 2, 10),           # non-finite y0
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, init=7),            # unknown start
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, init="coarse", coarse_points=-1),
        pp.make_problem("mol_heat_reaction", [0.01], [0.5] * 8, 0.0, 1.0, 2, 10, init="coarse"),
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, linearization=3),  # unknown linearisation
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, prior="matern", theta=0.0),  # length scale 0
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, prior="matern", theta=float("inf")),
        pp.make_problem("logistic", [], [0.1], 0.0, 1.0, 2, 10, prior=3),          # unknown prior
        # sigma-hat on the dense EK1 engine
        pp.make_problem("mol_heat_reaction", [0.01], [0.5] * 8, 0.0, 1.0, 2, 10, calibrate=True),
    ]
    for b in bad:
        with pytest.raises(pp.ParapnError) as e:
            pp.workspace_size(b)
        assert e.value.code == pp.EINVAL
        assert pp.last_error()


def test_no_cpu_fallback_without_library(tmp_path):
    """The binding refuses to run when the shared library is absent."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("pp_copy", os.path.join(ROOT, "paper_2310_01145_amd",
                                                                           "__init__.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with pytest.raises(ImportError):
        mod.load_library(str(tmp_path / "missing.so"))


def test_server_host_validation():
    """Server entry points reject bad arguments before any device work."""
    import paper_2310_01145_amd as pp

    L = pp.load_library()
    h = ctypes.c_void_p()
    assert L.parapn_server_create(ctypes.byref(h), None, 4, 0, None) == pp.EINVAL
    assert L.parapn_server_submit(None, None, 0, None, None) == pp.EINVAL
    assert L.parapn_server_step(None, None, None) == pp.EINVAL
    assert L.parapn_server_poll(None, None, 0, None) == pp.EINVAL
    assert L.parapn_server_stats(None, None, None, None, None) == pp.EINVAL
    L.parapn_server_destroy(None)
    t0 = L.parapn_server_clock()
    assert L.parapn_server_clock() >= t0
    # the admission footprint: linear in N, doubled elements in FP64
    f1 = pp.server_footprint("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 12, precision="fp32")
    f2 = pp.server_footprint("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 13, precision="fp32")
    f64 = pp.server_footprint("fhn", [0.2, 0.2, 3.0], [-1.0, 1.0], 0.0, 100.0, 3, 1 << 12, precision="fp64")
    assert 1.9 * f1 < f2 < 2.1 * f1 and 1.5 * f1 < f64 < 2.5 * f1
    # it covers at least the resident FP64 trajectory and the per-step scratch
    D, N = 8, 1 << 12
    assert f1 > (N + 1) * D * 8 + (N + 1) * (D * D + D) * 4
    with pytest.raises(pp.ParapnError) as e:
        pp.server_footprint("logistic", [], [0.1], 0.0, 1.0, 2, 0)
    assert e.value.code == pp.EINVAL


def test_dense_engine_host_checks():
    """Method-of-lines problems (the dense engine): workspace sizing follows
    the element layout (3 D^2 + 2 D filtering and 2 D^2 + D smoothing values
    per step, plus the covariance factors) and the field's argument checks."""
    import paper_2310_01145_amd as pp

    pp.load_library()
    y0 = [0.5] * 64
    w32 = pp.workspace_size(pp.make_problem("mol_heat_reaction", [0.01], y0, 0.0, 1.0, 2, 4096, precision="fp32"))
    w64 = pp.workspace_size(pp.make_problem("mol_heat_reaction", [0.01], y0, 0.0, 1.0, 2, 4096, precision="fp64"))
    D, N = 192, 4096
    per_step = 4 * (5 * D * D + 3 * D)  # FP32: A, C, J, E, L and b, e, g
    assert per_step * N < w32 < per_step * N + (2 << 30)  # + scratch slots and the trajectory
    # FP64 doubles the element arrays; the scratch slots take the same bytes
    # in both precisions (half as many, twice the size) and the trajectory is
    # FP64 in both
    assert abs((w64 - w32) - per_step * N) < 4096
    bad = [
        pp.make_problem("mol_heat_reaction", [0.01], [0.5, 0.5], 0.0, 1.0, 2, 10),              # d < 3
        pp.make_problem("mol_heat_reaction", [0.01], [0.5] * 100, 0.0, 1.0, 2, 10),             # D = 300 > 256
        pp.make_problem("mol_heat_reaction", [], [0.5] * 8, 0.0, 1.0, 2, 10),                   # no nu
        pp.make_problem("mol_heat_reaction", [-1.0], [0.5] * 8, 0.0, 1.0, 2, 10),               # nu < 0
        pp.make_problem("mol_heat_reaction", [0.01], [0.5] * 8, 0.0, 1.0, 2, 10, lm_sigma=0.1),  # damping
    ]
    for b in bad:
        with pytest.raises(pp.ParapnError) as e:
            pp.workspace_size(b)
        assert e.value.code == pp.EINVAL
    with pytest.raises(pp.ParapnError) as e:
        pp.server_footprint("mol_heat_reaction", [0.01], [0.5] * 8, 0.0, 1.0, 2, 10, precision="fp32")
    assert e.value.code == pp.EINVAL


def test_noalloc_entry_point_refuses_problems_beyond_its_scratch():
    """parapn_pararts_noalloc checks the size against its static scratch
    before touching the device (PARAPN_ENOMEM with a message)."""
    import paper_2310_01145_amd as pp

    L = pp.load_library()
    L.parapn_pararts_noalloc.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32] + \
        [ctypes.c_void_p] * 11
    L.parapn_pararts_noalloc.restype = ctypes.c_int
    fake = [ctypes.c_void_p(256)] * 6 + [ctypes.c_void_p(256), None, None, None, None]
    rc = L.parapn_pararts_noalloc(8, 2, 10_000_000, pp.FP32_SQRT, *fake)
    assert rc == pp.ENOMEM
    assert "static scratch" in pp.last_error()
    rc = L.parapn_pararts_noalloc(8, 2, 100, 7, *fake)
    assert rc == pp.EINVAL
