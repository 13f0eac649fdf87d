"""The C-ABI library loads and exports every function include/gacelle.h
declares; host-side helpers that need no GPU behave as documented."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gacelle.h")
LIB = os.path.join(ROOT, "paper_2511_22094_amd", "libgacelle.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(gc_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("gc_fit_askadam", "gc_mcmc", "gc_model_create", "gc_model_forward",
                 "gc_model_vjp", "gc_loss_vjp", "gc_tv", "gc_philox", "gc_server_create",
                 "gc_submit", "gc_wait", "gc_server_stats"):
        assert must in names
    assert len(names) >= 29


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (gc_\w+)", out))
    assert set(declared_functions()) <= exported


def test_host_only_entry_points(lib):
    from paper_2511_22094_amd import lib as load
    g = load()
    assert "gfx950" in g.gc_version()
    from paper_2511_22094_amd import build
    assert build.source_hash() in g.gc_version()
    assert g.gc_burnin_from_ratio(0.1, 25000) == 2500
    m = g.Model("gre3", te=[2.0 + 2 * i for i in range(24)])
    assert (m.n_params, m.n_meas_eff, m.is_complex) == (9, 48, True)
    assert m.param_names[3] == "T2s1"
    with pytest.raises(g.GcError) as e:
        g.Model("nexi", te=[1.0, 2.0])
    assert e.value.code == -2
    with pytest.raises(g.GcError) as e:
        g.Model("dwi2", bval=[1000.0])          # no directions
    assert e.value.code == -1
    with pytest.raises(g.GcError):
        g.Model("monoexp_t2s", te=[1.0, float("nan")])
    import numpy as np
    mask = np.zeros((3, 4, 5), np.uint8)
    mask[1, 2, 3] = mask[2, 0, 0] = 1
    assert g.gc_count_mask(mask) == 2
