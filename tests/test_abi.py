"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, reports sizes, and rejects bad arguments before any HIP call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "magx.h")


def _lib():
    from paper_2602_12242_amd import magx
    if not os.path.exists(magx.LIB_PATH):
        pytest.skip("libmagx.so not built")
    return magx, magx.load()


def test_exports_every_declared_symbol():
    magx, lib = _lib()
    decl = set(re.findall(r"\b(magx_[a-z_0-9]+)\s*\(", open(HEADER).read()))
    assert decl == set(magx.EXPORTS)
    for name in decl:
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    # sizes and field offsets as the C compiler lays out the header's structs
    import shutil
    import subprocess
    magx, _ = _lib()
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"magx_grid": magx.magx_grid, "magx_params": magx.magx_params,
               "magx_size_info": magx.magx_size_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "magx.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for f, _t in cls._fields_:
            lines.append(f'printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                 check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls)
        for f, _t in cls._fields_:
            assert int(out[f"{name}.{f}"]) == getattr(cls, f).offset


def test_sizes_of_workloads():
    magx, _ = _lib()
    s = magx.magx_sizes((512, 512, 32), (2.5e-9,) * 3, magx.F32)
    N = 512 * 512 * 32
    assert s["field_bytes"] == 3 * N * 4
    # [Hy][ntz][6][Hz][tz]: single precision with Pz = 64 takes 32-column
    # tiles (17 for Hx = 513) plus a copy of the Nyquist column in 16 + 1
    # such blocks along ky, double precision 16-column tiles (33)
    assert s["spectrum_bytes"] == (6 * 33 * 513 * (17 * 32) + 17 * 6 * 33 * 32) * 4
    assert s["tape_bytes_per_step"] == 28 * N * 4
    s64 = magx.magx_sizes((512, 512, 32), (2.5e-9,) * 3, magx.F64)
    assert s64["spectrum_bytes"] == 6 * 33 * 513 * (33 * 16) * 8
    # the large workload fits
    s = magx.magx_sizes((1024, 1024, 64), (3e-9,) * 3, magx.F32)
    assert s["workspace_bytes"] < 40e9


def test_batched_sizes_scale_with_the_batch():
    magx, lib = _lib()
    n, d = (256, 256, 16), (2e-9,) * 3
    s1 = magx.magx_sizes(n, d, magx.F32)
    for B in (1, 3, 8):
        sb = magx.magx_sizes(n, d, magx.F32, nbatch=B)
        # the spectrum and its build scratch are shared by the members
        assert sb["spectrum_bytes"] == s1["spectrum_bytes"]
        assert sb["init_scratch_bytes"] == s1["init_scratch_bytes"]
        assert sb["field_bytes"] == B * s1["field_bytes"]
        assert sb["tape_bytes_per_step"] == B * s1["tape_bytes_per_step"]
        assert sb["tape_bytes_extra"] == B * s1["tape_bytes_extra"]
        assert sb["workspace_bytes"] >= B * (s1["workspace_bytes"] - 4096)
    info = magx.magx_size_info()
    g = magx.make_grid(n, d)
    assert lib.magx_sizes_batched(ctypes.byref(g), 0, 0, ctypes.byref(info)) == -1
    assert lib.magx_sizes_batched(ctypes.byref(g), 0, -2, ctypes.byref(info)) == -1
    # the batch's spectral intermediates must stay below 2^31 elements
    g = magx.make_grid((1024, 1024, 64), (3e-9,) * 3)
    assert lib.magx_sizes_batched(ctypes.byref(g), 0, 1, ctypes.byref(info)) == 0
    assert lib.magx_sizes_batched(ctypes.byref(g), 0, 64, ctypes.byref(info)) == -2
    nul = ctypes.c_void_p(0)
    h = ctypes.c_void_p(12345)
    assert lib.magx_tensor_init_batched(ctypes.byref(h), ctypes.byref(g), 0, 2, nul, nul, nul) == -1
    assert h.value is None
    assert lib.magx_set_member_bias(nul, nul) == -1
    assert lib.magx_ctx_batch(nul) == -1


def test_sizes_at_the_limits():
    magx, _ = _lib()
    for dt in (magx.F32, magx.F64):
        # Pz = 1024 and Py = 4096 are the longest z and y transforms
        assert magx.magx_sizes((4, 4, 512), (1e-9,) * 3, dt)["field_bytes"] > 0
        assert magx.magx_sizes((4, 2048, 4), (1e-9,) * 3, dt)["field_bytes"] > 0
    assert magx.magx_sizes((2048, 4, 4), (1e-9,) * 3, magx.F32)["field_bytes"] > 0


@pytest.mark.parametrize("n,d,dt,code", [
    ((0, 4, 4), (1e-9,) * 3, 0, -1),
    ((4, 4, 4), (0.0, 1e-9, 1e-9), 0, -1),
    ((4, 4, 4), (1e-9,) * 3, 7, -3),
    ((5000, 4, 4), (1e-9,) * 3, 0, -2),
    ((4, 4, 2048), (1e-9,) * 3, 1, -2),
    ((4, 4, 1024), (1e-9,) * 3, 0, -2),
    ((4, 4, 1024), (1e-9,) * 3, 1, -2),
])
def test_sizes_rejects(n, d, dt, code):
    magx, lib = _lib()
    info = magx.magx_size_info()
    g = magx.make_grid(n, d)
    assert lib.magx_sizes(ctypes.byref(g), dt, ctypes.byref(info)) == code


def test_entry_points_reject_null_arguments_without_a_gpu():
    magx, lib = _lib()
    p = magx.make_params(8e5, A=1.3e-11)
    nul = ctypes.c_void_p(0)
    g = magx.make_grid((4, 4, 4), (1e-9,) * 3)
    h = ctypes.c_void_p(12345)
    assert lib.magx_tensor_init(ctypes.byref(h), ctypes.byref(g), 0, nul, nul, nul) == -1
    assert h.value is None
    # a spectrum that is not 16-byte aligned is refused before anything touches it
    h = ctypes.c_void_p(12345)
    odd = ctypes.c_void_p(0x10008)
    assert lib.magx_tensor_init(ctypes.byref(h), ctypes.byref(g), 1, odd, ctypes.c_void_p(0x20000), nul) == -1
    assert h.value is None
    assert lib.magx_heff(nul, nul, ctypes.byref(p), nul, nul, nul) == -1
    assert lib.magx_step(nul, nul, ctypes.byref(p), 1e-13, 1, nul, nul, nul) == -1
    assert lib.magx_heff_backward(nul, nul, ctypes.byref(p), nul, nul, nul, nul) == -1
    assert lib.magx_step_backward(nul, nul, 1, ctypes.byref(p), 1e-13, nul, nul, nul, nul) == -1
    assert lib.magx_llg_rhs(nul, nul, nul, ctypes.byref(p), nul, nul) == -1
    assert lib.magx_energy(nul, nul, ctypes.byref(p), nul, nul, nul) == -1
    assert lib.magx_heff_count(nul) == -1
    assert lib.magx_status(nul) == -1
    b = ctypes.c_double()
    assert lib.magx_memory_probe(nul, 0, nul, nul, ctypes.byref(b)) == -1
    assert lib.magx_step_static(nul, nul, ctypes.byref(p), 1e-13, 1, nul) == -1
    assert lib.magx_step_euler(nul, nul, ctypes.byref(p), 1e-13, 1, nul, nul) == -1
    assert lib.magx_step_mri(nul, nul, ctypes.byref(p), 1e-13, 1e-14, 1, nul, nul) == -1
    assert lib.magx_set_bias_schedule(nul, 0, None, None, 0.0) == -1
    assert lib.magx_set_ms_profile(nul, nul) == -1
    t = ctypes.c_double()
    assert lib.magx_get_time(nul, ctypes.byref(t)) == -1
    assert lib.magx_strerror(-2) == b"grid too large for the FFT passes"


def test_binding_wraps_every_entry_point():
    from paper_2602_12242_amd import magx
    for name in ("heff", "llg_rhs", "step", "step_static", "status", "step_mri", "step_euler", "set_bias_schedule", "heff_backward", "step_backward", "rollout_forward",
                 "rollout_backward", "energy", "set_member_bias", "set_ms_profile", "spectrum_array", "profile_start",
                 "profile_stop", "tape", "checkpoint_store", "field"):
        assert callable(getattr(magx.Context, name)), name
    assert isinstance(magx.Context.heff_count, property)


def test_context_requires_library(monkeypatch, tmp_path):
    from paper_2602_12242_amd import magx
    monkeypatch.setattr(magx, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        magx.load(str(tmp_path / "nope.so"))
