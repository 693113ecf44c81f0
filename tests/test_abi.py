"""The C ABI on the host: symbols, struct layout and argument validation.

No test here launches GPU work; every call below returns before the first
HIP call (validation happens first by contract).
"""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2404_04441_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wave.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(L.LIB_PATH):
        from paper_2404_04441_amd.build import build
        build()
    return L.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wave_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(L.EXPORTS)


def test_params_struct_layout_matches_c(tmp_path):
    src = tmp_path / "layout.c"
    fields = [f for f, _ in L.WaveParams._fields_]
    body = "\n".join(f'printf("{f} %zu\\n", offsetof(wave_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "wave.h"\n'
                   'int main(void){' + body + 'printf("size %zu\\n", sizeof(wave_params));return 0;}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(L.WaveParams, f).offset, f
    assert int(out["size"]) == ctypes.sizeof(L.WaveParams)


def _params(lib, **kw):
    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    p.nx, p.ny, p.nz = 16, 12, 10
    p.dx = p.dy = p.dz = 10.0
    p.dt = 1e-4
    for k, v in kw.items():
        if k == "src":
            p.src[0], p.src[1], p.src[2] = v
        else:
            setattr(p, k, v)
    return p


def _bytes(lib, p):
    b = ctypes.c_size_t()
    rc = lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b))
    return rc, b.value


def test_workspace_bytes(lib):
    rc, b32 = _bytes(lib, _params(lib))
    assert rc == 0 and b32 % 256 == 0
    N = 16 * 12 * 10
    assert b32 >= 3 * 4 * N  # m and two float32 fields
    rc, b16 = _bytes(lib, _params(lib, storage=L.WAVE_F16))
    assert rc == 0 and b16 < b32
    rc, badj = _bytes(lib, _params(lib, adjoint=1, nt_max=100))
    # 10 steps per checkpoint: 9 checkpoint pairs + 12 segment slots + 3 adjoint fields
    assert rc == 0 and badj - b32 >= 4 * N * (2 * 9 + 12 + 3)
    # fields the step kernel touches carry 15 zero planes past nz
    rc, b40 = _bytes(lib, _params(lib, nz=40))
    assert rc == 0 and b40 - b32 >= 3 * 4 * 16 * 12 * 30


def test_cpml_workspace(lib):
    # psi and zeta slabs of W nodes per face pair on each axis (grid 16 x 12 x 10)
    rc, b0 = _bytes(lib, _params(lib))
    rc1, b1 = _bytes(lib, _params(lib, cpml_width=3))
    assert rc == 0 and rc1 == 0
    W2 = 6
    slabs = 4 * 2 * (10 * 12 * W2 + 10 * W2 * 16 + W2 * 12 * 16)
    assert b1 - b0 >= slabs + 4 * 2 * (16 + 12 + 10)


def test_cache_hint_accepted(lib):
    assert _bytes(lib, _params(lib, cache_hint=1))[0] == 0
    assert _bytes(lib, _params(lib, cache_hint=1, variant=12, nx=16))[0] == 0
    assert _bytes(lib, _params(lib, cache_hint=1, adjoint=1, nt_max=10))[0] == 0
    assert _bytes(lib, _params(lib, cache_hint=1, storage=L.WAVE_F16))[0] == 0


def test_plane_size_limit(lib):
    # at most 2^24 nodes per xy plane (buffer offsets of a z-chunk stay below 2^31 bytes)
    assert _bytes(lib, _params(lib, nx=4096, ny=4096, nz=1))[0] == 0
    assert _bytes(lib, _params(lib, nx=4097, ny=4096, nz=1))[0] == L.WAVE_EINVAL


@pytest.mark.parametrize("kw", [
    dict(nx=0), dict(nz=-1), dict(dt=0.0), dict(dx=float("nan")), dict(storage=3),
    dict(src=(16, 0, 0)), dict(src=(0, -1, 0)), dict(sponge_width=-1), dict(sponge_alpha=-0.1),
    dict(adjoint=1, nt_max=0), dict(adjoint=1, nt_max=10, storage=L.WAVE_F16), dict(variant=99),
    dict(zchunk=-2), dict(graph_steps=-1), dict(tune=2),
    dict(cpml_width=-1), dict(cpml_width=3, sponge_width=2), dict(cpml_width=3, storage=L.WAVE_F16),
    dict(cpml_width=3, adjoint=1, nt_max=10), dict(cpml_width=6), dict(cpml_width=3, cpml_reflection=0.0),
    dict(cpml_width=3, cpml_reflection=1.5), dict(cpml_width=3, cpml_f0=-1.0),
    dict(cache_hint=2), dict(cache_hint=-1),
    dict(cache_hint=1, cpml_width=3), dict(cache_hint=1, variant=14),
])
def test_invalid_params_rejected(lib, kw):
    rc, _ = _bytes(lib, _params(lib, **kw))
    assert rc == L.WAVE_EINVAL


def test_receivers_validated(lib):
    rec = (ctypes.c_int32 * 6)(1, 2, 3, 16, 0, 0)  # second receiver outside in x
    p = _params(lib, nrec=2)
    p.rec = ctypes.cast(rec, ctypes.POINTER(ctypes.c_int32))
    assert _bytes(lib, p)[0] == L.WAVE_EINVAL
    p = _params(lib, nrec=2)  # null pointer with nrec > 0
    assert _bytes(lib, p)[0] == L.WAVE_EINVAL


def test_create_checks_before_any_gpu_call(lib):
    p = _params(lib)
    rc, need = _bytes(lib, p)
    h = ctypes.c_void_p()
    fake = 1 << 20  # never dereferenced: every call below fails validation first
    assert lib.wave_create(ctypes.byref(p), fake, fake, need - 256, None, ctypes.byref(h)) == L.WAVE_ENOSPC
    assert lib.wave_create(ctypes.byref(p), fake, fake + 8, need, None, ctypes.byref(h)) == L.WAVE_EINVAL
    assert lib.wave_create(ctypes.byref(p), None, fake, need, None, ctypes.byref(h)) == L.WAVE_EINVAL
    assert lib.wave_create(ctypes.byref(p), fake, fake, need, None, None) == L.WAVE_EINVAL
    bad = _params(lib, nx=0)
    assert lib.wave_create(ctypes.byref(bad), fake, fake, need, None, ctypes.byref(h)) == L.WAVE_EINVAL


def test_null_context_calls(lib):
    n = ctypes.c_int32()
    f = ctypes.c_uint32()
    assert lib.wave_step(None, 1, None, None) == L.WAVE_EINVAL
    assert lib.wave_run(None, 1, None, None) == L.WAVE_EINVAL
    assert lib.wave_reset(None) == L.WAVE_EINVAL
    assert lib.wave_adjoint(None, 1, None, None, None) == L.WAVE_EINVAL
    assert lib.wave_read_field(None, 0, None) == L.WAVE_EINVAL
    assert lib.wave_write_field(None, 0, None) == L.WAVE_EINVAL
    assert lib.wave_time_index(None, ctypes.byref(n)) == L.WAVE_EINVAL
    assert lib.wave_sync_status(None, ctypes.byref(f)) == L.WAVE_EINVAL
    assert lib.wave_destroy(None) == L.WAVE_EINVAL
    assert lib.wave_workspace_bytes(None, None) == L.WAVE_EINVAL
    out = (ctypes.c_int32 * 3)()
    assert lib.wave_tiling(None, out) == L.WAVE_EINVAL


def test_params_defaults(lib):
    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    assert p.tune == 1 and p.cache_hint == 0 and p.variant == 0 and p.zchunk == 0
    assert p.storage == L.WAVE_F32 and p.src[0] < 0 and p.cpml_width == 0


def test_status_strings_and_variants(lib):
    for code in (0, -1, -2, -3, -4, -5):
        assert L.status_string(code)
    assert L.status_string(-77) == "unknown status"
    assert lib.wave_variant_count() >= 1


def test_variant_info_and_shape_validation(lib):
    n = lib.wave_variant_count()
    info = (ctypes.c_int32 * 5)()
    families = set()
    for v in range(n):
        assert lib.wave_variant_info(v, info) == 0
        fam, by, ry, pd, vec = list(info)
        families.add(fam)
        assert fam in (0, 1, 2, 3, 4) and by >= 1 and ry >= 1 and pd >= 1 and vec in (1, 2, 4)
        if fam in (0, 3):
            assert 9 % pd == 0 and 8 * ry <= 64
        if fam == 4:  # the two-steps-per-pass kernel: only with time_block = 2, float32 forward
            assert _bytes(lib, _params(lib, variant=v, nx=16))[0] == L.WAVE_EINVAL
            assert _bytes(lib, _params(lib, variant=v, nx=18, time_block=2))[0] == 0
            assert _bytes(lib, _params(lib, variant=v, time_block=2, storage=L.WAVE_F16))[0] == L.WAVE_EINVAL
            assert _bytes(lib, _params(lib, variant=v, time_block=2, adjoint=1, nt_max=10))[0] == L.WAVE_EINVAL
            assert _bytes(lib, _params(lib, variant=v, time_block=2, graph_steps=6))[0] == L.WAVE_EINVAL
            continue
        # nx = 16 accepts every lane width; nx = 18 (even, not a multiple of 4) rejects vec 4
        assert _bytes(lib, _params(lib, variant=v, nx=16))[0] == 0
        assert (_bytes(lib, _params(lib, variant=v, nx=18))[0] == 0) == (vec != 4)
        # the study families (3D-blocked, semi-stencil) are float32 forward only
        rc16 = _bytes(lib, _params(lib, variant=v, nx=16, storage=L.WAVE_F16))[0]
        rcadj = _bytes(lib, _params(lib, variant=v, nx=16, adjoint=1, nt_max=10))[0]
        assert (rc16 == 0) == (fam == 0) and (rcadj == 0) == (fam == 0)
        # a one-step shape with time_block = 2 is refused (variant 0, automatic, is not a shape)
        assert (_bytes(lib, _params(lib, variant=v, nx=16, time_block=2))[0] == L.WAVE_EINVAL) == (v != 0)
    assert families == {0, 1, 2, 3, 4}
    # time_block = 2 adds two float32 fields to the workspace
    one = _bytes(lib, _params(lib))
    two = _bytes(lib, _params(lib, time_block=2))
    assert one[0] == two[0] == 0 and two[1] > one[1]
    assert lib.wave_variant_info(n, info) == L.WAVE_EINVAL
    assert lib.wave_variant_info(-1, info) == L.WAVE_EINVAL
    assert lib.wave_variant_info(0, None) == L.WAVE_EINVAL


def test_static_workspace_size_checked_before_the_device(lib):
    """wave_create_static refuses a workspace larger than its static array
    (and graph replay) without touching a GPU."""
    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    p.nx = p.ny = p.nz = 512
    p.dt = 1e-4
    b = ctypes.c_size_t()
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == L.WAVE_OK
    assert b.value > L.WAVE_STATIC_BYTES
    h = ctypes.c_void_p()
    fake_vel = ctypes.c_void_p(256)  # never dereferenced: the size check comes first
    assert lib.wave_create_static(ctypes.byref(p), fake_vel, None, ctypes.byref(h)) == L.WAVE_ENOSPC
    p.nx = p.ny = p.nz = 16
    p.graph_steps = 4
    assert lib.wave_create_static(ctypes.byref(p), fake_vel, None, ctypes.byref(h)) == L.WAVE_EINVAL
    assert lib.wave_create_static(None, fake_vel, None, ctypes.byref(h)) == L.WAVE_EINVAL
    assert not h.value


def test_model_bits_validation(lib):
    """16-bit model codes exist for 16-bit wavefield storage only."""
    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    p.nx = p.ny = p.nz = 16
    p.dt = 1e-4
    b = ctypes.c_size_t()
    ws32 = ctypes.c_size_t()
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(ws32)) == L.WAVE_OK
    p.model_bits = 16
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == L.WAVE_EINVAL  # float32 storage
    p.storage = L.WAVE_F16
    p.model_bits = 8
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == L.WAVE_EINVAL
    p.model_bits = 32
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == L.WAVE_OK
    full = b.value
    p.model_bits = 16
    assert lib.wave_workspace_bytes(ctypes.byref(p), ctypes.byref(b)) == L.WAVE_OK
    assert b.value < full  # m as 2-byte codes


def test_stability_limit_on_the_host(lib):
    """The time-step limit wave_create enforces, as a host function: against
    the oracle's leapfrog stability bound (dense-operator pinned) on a cubic
    grid, the anisotropic formula, and the reading of "CFL 0.5" the workloads
    use (half the limit)."""
    import oracle
    from synth import COURANT

    p = L.WaveParams()
    lib.wave_params_init(ctypes.byref(p))
    p.dx = p.dy = p.dz = 10.0
    dt = ctypes.c_double()
    assert lib.wave_stable_dt(ctypes.byref(p), 4500.0, ctypes.byref(dt)) == L.WAVE_OK
    assert abs(dt.value * 4500.0 / 10.0 - oracle.stability_courant(3)) < 1e-12
    assert abs(COURANT / (dt.value * 4500.0 / 10.0) - 0.5) < 1e-12
    p.dx, p.dy, p.dz = 10.0, 12.0, 9.0
    assert lib.wave_stable_dt(ctypes.byref(p), 3000.0, ctypes.byref(dt)) == L.WAVE_OK
    peak = float(oracle.symbol_peak(4))
    want = 2.0 / (3000.0 * (peak * (1 / 100 + 1 / 144 + 1 / 81)) ** 0.5)
    assert abs(dt.value / want - 1) < 1e-12
    assert lib.wave_stable_dt(ctypes.byref(p), 0.0, ctypes.byref(dt)) == L.WAVE_EINVAL
    assert lib.wave_stable_dt(ctypes.byref(p), float("nan"), ctypes.byref(dt)) == L.WAVE_EINVAL
    assert lib.wave_stable_dt(None, 3000.0, ctypes.byref(dt)) == L.WAVE_EINVAL
