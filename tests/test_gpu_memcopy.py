"""GPU tests of rl_memcopy (copies between memory contexts, Sec. VII-A,
with the variants for partially overlapping arrays that insertion and
deletion use): the result must equal the plain definition of a move,
dst[:] = a copy of src[:] taken before any byte is written (numpy slices
copied out first), byte for byte."""
import numpy as np
import pytest

import paper_2511_04853_amd as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _rand(n, seed):
    return np.random.default_rng(seed).integers(0, 256, size=n, dtype=np.uint8)


@pytest.mark.parametrize("nbytes,src_off,dst_off", [(1, 0, 0), (15, 3, 5), (4096, 0, 0), (100_003, 7, 7),
                                                    (1 << 20, 16, 32), (3_000_001, 1, 9)])
def test_disjoint_device_copy(nbytes, src_off, dst_off):
    h = _rand(nbytes + 64, nbytes)
    src = torch.from_numpy(h).cuda()
    dst = torch.full((nbytes + 64,), 0xCD, dtype=torch.uint8, device="cuda")
    P.memcopy(dst.data_ptr() + dst_off, "device", src.data_ptr() + src_off, "device", nbytes)
    torch.cuda.synchronize()
    want = np.full(nbytes + 64, 0xCD, np.uint8)
    want[dst_off:dst_off + nbytes] = h[src_off:src_off + nbytes]
    assert np.array_equal(dst.cpu().numpy(), want)


@pytest.mark.parametrize("nbytes,shift", [(1000, 1), (1000, -1), (1 << 20, 4096), (1 << 20, -4096),
                                          (5_000_003, 17), (5_000_003, -17),
                                          # several 64 MiB bands through scratch
                                          (150 << 20, 4096), (150 << 20, -4096),
                                          # shifts of 64 MiB and more: direct bands
                                          (200 << 20, 70 << 20), (200 << 20, -(70 << 20))])
def test_overlapping_device_move(nbytes, shift):
    total = nbytes + abs(shift) + 32
    h = _rand(total, abs(shift) + nbytes)
    buf = torch.from_numpy(h).cuda()
    src = 16 if shift > 0 else 16 + abs(shift)
    dst = src + shift
    P.memcopy(buf.data_ptr() + dst, "device", buf.data_ptr() + src, "device", nbytes)
    torch.cuda.synchronize()
    want = h.copy()
    want[dst:dst + nbytes] = h[src:src + nbytes].copy()
    got = buf.cpu().numpy()
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:5]}"


@pytest.mark.parametrize("space", ["pinned", "host"])
def test_host_device_round_trip(space):
    n = 3_000_017
    h = _rand(n, 5)
    src = torch.from_numpy(h.copy())
    if space == "pinned":
        src = src.pin_memory()
    dev = torch.empty(n, dtype=torch.uint8, device="cuda")
    back = torch.zeros(n, dtype=torch.uint8)
    if space == "pinned":
        back = back.pin_memory()
    P.memcopy(dev, "device", src, space, n)
    P.memcopy(back, space, dev, "device", n)
    torch.cuda.synchronize()
    assert np.array_equal(back.numpy(), h)


def test_host_to_host_move_overlapping():
    h = _rand(10_000, 6)
    buf = h.copy()
    P.memcopy(buf.ctypes.data + 100, "host", buf.ctypes.data, "host", 9_000)
    want = h.copy()
    want[100:9100] = h[0:9000].copy()
    assert np.array_equal(buf, want)


def test_zero_bytes_and_bad_arguments():
    import ctypes
    t = torch.zeros(16, dtype=torch.uint8, device="cuda")
    P.memcopy(t, "device", t, "device", 0)
    st = P.lib().rl_memcopy(None, 0, ctypes.c_void_p(t.data_ptr()), 0, 16, P.stream_ptr(None))
    assert st == P.RL_EINVAL
    st = P.lib().rl_memcopy(ctypes.c_void_p(t.data_ptr()), 7, ctypes.c_void_p(t.data_ptr()), 0, 16, P.stream_ptr(None))
    assert st == P.RL_EINVAL
