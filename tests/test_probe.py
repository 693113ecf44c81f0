"""The benchmark's HIP stream probes (libwave_probe.so): exports and argument
checks on the CPU; on the GPU, each probe's output element by element on a
ragged size (the last workgroup partly past the end)."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "paper_2404_04441_amd", "libwave_probe.so")
HIP_ERROR_INVALID_VALUE = 1


@pytest.fixture(scope="module")
def probe():
    if not os.path.exists(PROBE):
        from paper_2404_04441_amd.build import build
        build()
    L = ctypes.CDLL(PROBE)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.probe_stream_3r1w.argtypes = [vp, vp, vp, vp, sz, vp]
    L.probe_copy.argtypes = [vp, vp, sz, vp]
    L.probe_stream_16bit.argtypes = [vp, vp, vp, vp, vp, sz, ctypes.c_int, vp]
    return L


def test_probe_exports_and_argument_checks(probe):
    # sizes that are not a multiple of 4 and null pointers are refused before any launch
    fake = ctypes.c_void_p(256)
    assert probe.probe_stream_3r1w(fake, fake, fake, fake, 6, None) == HIP_ERROR_INVALID_VALUE
    assert probe.probe_copy(None, fake, 8, None) == HIP_ERROR_INVALID_VALUE
    assert probe.probe_stream_16bit(fake, fake, fake, fake, fake, 10, 0, None) == HIP_ERROR_INVALID_VALUE
    assert probe.probe_stream_16bit(fake, None, fake, fake, fake, 8, 1, None) == HIP_ERROR_INVALID_VALUE


@pytest.mark.gpu
def test_probe_outputs(probe):
    torch = pytest.importorskip("torch")
    dev = torch.device("cuda")
    st = torch.cuda.current_stream().cuda_stream
    rng = np.random.default_rng(5)
    n = 4 * 1025 * 3 + 4  # groups past a whole number of workgroups
    print(f"case: stream probes, n = {n}", flush=True)
    # small integers: every float32 result is exact
    a, b, c = (rng.integers(-64, 64, n).astype(np.float32) for _ in range(3))
    ta, tb, tc = (torch.from_numpy(x).to(dev) for x in (a, b, c))
    td = torch.full((n + 64,), 7.0, device=dev)
    assert probe.probe_stream_3r1w(ta.data_ptr(), tb.data_ptr(), tc.data_ptr(), td.data_ptr(), n, st) == 0
    torch.cuda.synchronize()
    d = td.cpu().numpy()
    assert np.array_equal(d[:n], a + b * c) and np.all(d[n:] == 7.0)
    td.fill_(7.0)
    assert probe.probe_copy(ta.data_ptr(), td.data_ptr(), n, st) == 0
    torch.cuda.synchronize()
    d = td.cpu().numpy()
    assert np.array_equal(d[:n], a) and np.all(d[n:] == 7.0)

    for m16 in (0, 1):
        ha, hv = (rng.integers(0, 2 ** 16, n).astype(np.uint16) for _ in range(2))
        hm = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)  # n words; codes use the first half
        ga, gv = (torch.from_numpy(x.view(np.int16)).to(dev) for x in (ha, hv))
        gm = torch.from_numpy(hm.view(np.int32)).to(dev)
        gao = torch.full((n + 64,), 3, dtype=torch.int16, device=dev)
        gvo = torch.full((n + 64,), 3, dtype=torch.int16, device=dev)
        assert probe.probe_stream_16bit(ga.data_ptr(), gv.data_ptr(), gm.data_ptr(), gao.data_ptr(), gvo.data_ptr(),
                                        n, m16, st) == 0
        torch.cuda.synchronize()
        wa, wv = ha.view(np.uint32).reshape(-1, 2), hv.view(np.uint32).reshape(-1, 2)
        if m16:
            wm = hm[: n // 2].reshape(-1, 2)
        else:
            w4 = hm.reshape(-1, 4)
            wm = np.stack([w4[:, 0] ^ w4[:, 2], w4[:, 1] ^ w4[:, 3]], 1)
        ao = gao.cpu().numpy().view(np.uint16)
        vo = gvo.cpu().numpy().view(np.uint16)
        assert np.array_equal(ao[:n].view(np.uint32).reshape(-1, 2), wa ^ wm)
        assert np.array_equal(vo[:n].view(np.uint32).reshape(-1, 2), wv + wm)  # wrapping add per word
        assert np.all(ao[n:] == 3) and np.all(vo[n:] == 3)
        # V updated in place, as the benchmark runs it
        assert probe.probe_stream_16bit(ga.data_ptr(), gv.data_ptr(), gm.data_ptr(), gao.data_ptr(), gv.data_ptr(),
                                        n, m16, st) == 0
        torch.cuda.synchronize()
        assert np.array_equal(gv.cpu().numpy().view(np.uint16).view(np.uint32).reshape(-1, 2), wv + wm)
