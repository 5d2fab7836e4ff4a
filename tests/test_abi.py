"""CPU checks of the boundary: libsvf.so loads and exports every function that
include/svf.h declares; the host-only entry point answers without a GPU."""
import ctypes as C
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def declared_functions():
    text = (ROOT / "include" / "svf.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(svf_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_path():
    names = declared_functions()
    for n in ["svf_filter", "svf_preintegrate", "svf_scale_map", "svf_create", "svf_destroy", "svf_filter_batch"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1003_2022_amd as P

    L = P.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_workspace_bytes_host_only():
    import paper_1003_2022_amd as P

    img = P.svf_image(None, P.SVF_F32, 1, 4096, 4096, 4096)
    o = P.default_opts()
    n = P.svf_workspace_bytes(img, 4, 2, o)
    # scales 16 B/px + one window per 256-tile of (256 + 2*128 + 5)^2 doubles
    assert n >= 4096 * 4096 * 16 + 256 * (517 ** 2) * 8
    with pytest.raises(P.SvfError):
        P.svf_workspace_bytes(img, 3, 2, o)     # N != 4
    with pytest.raises(P.SvfError):
        P.svf_workspace_bytes(img, 4, 4, o)     # order out of range


def test_default_opts():
    import paper_1003_2022_amd as P

    o = P.default_opts()
    assert o.preint == P.SVF_PRE_F64 and o.fd_fp32 == 0 and o.eps_px2 == 0.25 and o.max_reach_px == 128
    assert o.bands == 0 and o.boundary == P.SVF_BOUNDARY_ZERO


def test_workspace_bytes_rejects_bad_boundary():
    import paper_1003_2022_amd as P

    img = P.svf_image(None, P.SVF_F32, 1, 64, 64, 64)
    for b in (P.SVF_BOUNDARY_REPLICATE, P.SVF_BOUNDARY_SYMMETRIC):
        assert P.svf_workspace_bytes(img, 4, 1, P.default_opts(boundary=b)) > 0
    for b in (-1, 3):
        with pytest.raises(P.SvfError):
            P.svf_workspace_bytes(img, 4, 1, P.default_opts(boundary=b))
