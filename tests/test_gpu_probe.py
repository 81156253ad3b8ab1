"""The bandwidth probe (naj_bandwidth_probe): the copy mode copies exactly, every mode reports a time,
and invalid arguments are refused before any device work."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def naj():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2407_03272_amd import naj as N
    N.load()
    return N


def test_probe_modes(naj):
    print("[gpu-case] bandwidth probe, 64 MiB", flush=True)
    for mode in (0, 1, 2):
        r = naj.bandwidth_probe(mode, 64 << 20, 3)
        assert r["ms"] > 0 and r["gbps"] > 0
        if mode == 1:
            assert r["copy_exact"]


def test_probe_copy_of_a_ragged_size(naj):
    import torch
    n = (1 << 20) + 3                       # not a multiple of the grid's sweep
    src = torch.arange(2 * n, dtype=torch.float64, device="cuda:0")
    dst = torch.zeros_like(src)
    ms = ctypes.c_double()
    st = naj.load().naj_bandwidth_probe(1, ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                                        src.numel() * 8, 2, ctypes.byref(ms), None)
    torch.cuda.synchronize()
    assert st == 0 and torch.equal(src, dst)


def test_probe_write_of_a_ragged_size(naj):
    """Mode 2 writes word i of 16 bytes as (i, i+1, i+2, i+3) over every full block and the partial one."""
    import torch
    n16 = 3 * 1024 + 5                      # three full 16 KB blocks and a partial one
    dst = torch.zeros(4 * n16, dtype=torch.int32, device="cuda:0")
    ms = ctypes.c_double()
    st = naj.load().naj_bandwidth_probe(2, None, ctypes.c_void_p(dst.data_ptr()), n16 * 16, 1, ctypes.byref(ms),
                                        None)
    torch.cuda.synchronize()
    assert st == 0
    i = torch.arange(n16, dtype=torch.int64, device="cuda:0")
    want = torch.stack([i, i + 1, i + 2, i + 3], dim=1).reshape(-1).to(torch.int32)
    assert torch.equal(dst, want)


def test_probe_rejects_bad_arguments(naj):
    ms = ctypes.c_double()
    lib = naj.load()
    assert lib.naj_bandwidth_probe(3, None, None, 1024, 1, ctypes.byref(ms), None) == naj.NAJ_EINVAL
    assert lib.naj_bandwidth_probe(2, None, None, 1024, 1, ctypes.byref(ms), None) == naj.NAJ_EINVAL
    assert lib.naj_bandwidth_probe(0, None, None, 1000, 1, ctypes.byref(ms), None) == naj.NAJ_EINVAL
