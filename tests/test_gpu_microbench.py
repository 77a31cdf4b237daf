"""The ceiling probes (cfs_microbench) do the work they report: the copy
copies, every random atomic add lands once, atomic minima only lower
values, the Philox probe's blocks are the generator's, and the run reads read
what their address sequence names."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2606_02226_amd import api as _api
    return _api


def _dev():
    return torch.device("cuda:0")


def test_copy(api):
    buf = torch.empty(1 << 22, dtype=torch.uint8, device=_dev())
    half = buf.numel() // 2
    buf[:half] = torch.randint(0, 256, (half,), dtype=torch.uint8, device=_dev())
    done = api.microbench("copy", buf)
    torch.cuda.synchronize()
    assert done == buf.numel()
    assert torch.equal(buf[:half], buf[half:])


def test_device_atomics(api):
    buf = torch.zeros(1 << 20, dtype=torch.uint8, device=_dev())
    done = api.microbench("dev_add_u32", buf, ops=1 << 22)
    torch.cuda.synchronize()
    counts = buf.view(torch.int32).cpu().numpy().view(np.uint32).astype(np.int64)
    assert done >= 1 << 22 and counts.sum() == done
    assert np.count_nonzero(counts) > 0.9 * counts.size   # spread over the set
    buf.fill_(0xFF)
    done = api.microbench("dev_min_u64", buf, ops=1 << 22)
    torch.cuda.synchronize()
    keys = buf.view(torch.int64).cpu().numpy().view(np.uint64)
    assert done >= 1 << 22 and np.count_nonzero(keys != np.uint64(2**64 - 1)) > 0.9 * keys.size


def test_lds_atomics(api):
    for kind in ("lds_add_u32", "lds_add_u64", "lds_min_u64"):
        buf = torch.zeros(4096, dtype=torch.uint8, device=_dev())
        done = api.microbench(kind, buf, ops=1 << 24)
        torch.cuda.synchronize()
        assert done >= 1 << 24
        w = buf.view(torch.int32 if kind == "lds_add_u32" else torch.int64)[:512]
        assert torch.count_nonzero(w).item() == 512


def test_philox_blocks(api, orc):
    lanes = 4096 * 256
    buf = torch.zeros(lanes * 4, dtype=torch.uint8, device=_dev())
    done = api.microbench("philox", buf, ops=lanes * 3)
    torch.cuda.synchronize()
    assert done == lanes * 3
    got = buf.view(torch.int32).cpu().numpy().view(np.uint32)
    seed = 0x9ABCDEF0 << 32 | 0x12345678
    for g in (0, 1, 777, lanes - 1):
        ref = 0
        for i in range(3):
            b = orc.philox_many(seed, np.array([[g, i, 0, 0]], np.uint32))[0]
            ref ^= int(b[0] ^ b[1] ^ b[2] ^ b[3])
        assert int(got[g]) == ref, g


@pytest.mark.parametrize("kind,lg", [("runs_128", 3), ("runs_512", 5), ("runs_2048", 7)])
def test_run_reads(api, kind, lg):
    """Each lane's word is the xor of the 16-byte vectors it read: run
    starts from its group's congruential sequence, scaled to the buffer by a
    high multiply, and the lane's vector within the run."""
    lanes, head = 4096 * 256, 4 << 20
    nbytes = head + (16 << 20)
    buf = torch.zeros(nbytes, dtype=torch.uint8, device=_dev())
    nw = (nbytes - head) // 4
    words = (np.arange(nw, dtype=np.uint64) * 2654435761 % (1 << 32)).astype(np.uint32)
    buf[head:] = torch.from_numpy(words.view(np.uint8)).to(_dev())
    ops = 1 << 18
    done = api.microbench(kind, buf, ops=ops)
    torch.cuda.synchronize()
    groups = lanes >> lg
    pg = -(-ops // groups)
    pg = (pg + 3) // 4 * 4
    assert done == groups * pg * (16 << lg)
    got = buf[:lanes * 4].view(torch.int32).cpu().numpy().view(np.uint32)
    vec = words.reshape(-1, 4)
    n_start = vec.shape[0] - (1 << lg) + 1
    for g in (0, 1, (1 << lg) + 3, lanes - 1):
        h = ((g >> lg) * 0x9E3779B9 + 0x7F4A7C15) % (1 << 32)
        acc = 0
        for _ in range(pg):
            h = (h * 1664525 + 1013904223) % (1 << 32)
            v = vec[((h * n_start) >> 32) + (g & ((1 << lg) - 1))]
            acc ^= int(v[0] ^ v[1] ^ v[2] ^ v[3])
        assert int(got[g]) == acc, g
