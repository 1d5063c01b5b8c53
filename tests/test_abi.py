"""The C-ABI library loads and exports every entry point the public header
declares; the Python layer refuses to run without a GPU (no CPU fallback)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(rr_[a-z0-9_]+)\s*\(", txt))
    return names


def test_header_declares_core_entry_points():
    names = _declared()
    for n in ("rr_create", "rr_destroy", "rr_scene_upload", "rr_set_array", "rr_set_chirp",
              "rr_trace", "rr_synthesize"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_2307_15412_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        from paper_2307_15412_amd import build
        build.build()
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rr_[a-z0-9_]+)\b", out))
    missing = _declared() - exported
    assert not missing, missing
    lib = pkg.load_library()
    assert lib.rr_version().startswith(b"radray")
    # thread-local message of the last failing call (earlier tests in the same
    # process may have left one)
    assert isinstance(lib.rr_last_error(), bytes)


def test_no_gpu_no_fallback():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    import paper_2307_15412_amd as pkg
    with pytest.raises(RuntimeError):
        pkg.Context(0)


def test_invalid_args_rejected_without_device():
    """Entry points reject NULL handles with RR_EINVAL before touching HIP."""
    import ctypes as C
    import paper_2307_15412_amd as pkg
    lib = pkg.load_library()
    assert lib.rr_create(0, None, None) == pkg.binding.RR_EINVAL
    assert lib.rr_trace(None, None, None) == pkg.binding.RR_EINVAL
    assert lib.rr_synthesize(None, 0, 0, None, 0, None, 0) == pkg.binding.RR_EINVAL
    assert b"NULL" in lib.rr_last_error() or b"null" in lib.rr_last_error().lower()


def test_output_tensors_checked_before_the_library_sees_them():
    """Output tensors reach the library as bare addresses: a host tensor, a
    wrong dtype, a strided view or a short buffer is refused in the binding."""
    import torch
    from paper_2307_15412_amd.binding import check_out
    dev = torch.device("cuda", 0)
    host = torch.zeros(16, dtype=torch.complex64)
    with pytest.raises(ValueError):
        check_out(host, dev, torch.complex64, 16)
    with pytest.raises(ValueError):
        check_out(host, torch.device("cpu"), torch.complex64, 17)
    with pytest.raises(ValueError):
        check_out(host, torch.device("cpu"), torch.float32, 16)
    with pytest.raises(ValueError):
        check_out(torch.zeros((4, 8), dtype=torch.complex64)[:, ::2], torch.device("cpu"),
                  torch.complex64, 16)
    check_out(host, torch.device("cpu"), torch.complex64, 16)


def test_new_entry_points_reject_null_handles():
    """Per-face alpha, vertex update, BVH export, imaging, casting pieces,
    batch alpha and the batch's engine plan refuse a NULL handle before
    touching HIP."""
    import ctypes as C
    import paper_2307_15412_amd as pkg
    lib = pkg.load_library()
    E = pkg.binding.RR_EINVAL
    n = C.c_int64()
    assert lib.rr_scene_set_alpha(None, None, 0, 0) == E
    assert lib.rr_scene_update_vertices(None, None, 0) == E
    assert lib.rr_get_bvh_nodes(None, None, 0, C.byref(n)) == E
    assert lib.rr_backproject(None, None, 0, None, None, 0, 0) == E
    assert lib.rr_max_projection(None, None, None, None, C.c_float(-15.0)) == E
    assert lib.rr_set_casting(None, 1e-3, 4) == E
    assert lib.rr_casting_pieces(None, None, C.byref(n)) == E
    pkg.binding._declare_batch(lib)
    assert lib.rr_batch_set_alpha(None, 0, None, 0, 0) == E
    assert lib.rr_batch_set_engine(None, 0, 0, 0) == E
    assert lib.rr_batch_get_plan(None, None, None) == E
    assert lib.rr_last_error() != b""
