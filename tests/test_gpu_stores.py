"""GPU parity with values of direct destinations stored non-temporally and
with ordinary stores (the plan's default and the batch tuner's other
choice): every layout pair of single conversions, the single-pass jagged
kernel, and a batch with fan-out groups, against the oracle byte for byte."""
import pytest

import paper_2511_04853_amd as P
import workloads as W
from tests.test_gpu_fanout import _run, _shared_source_items
from tests.test_gpu_parity import _check, _kinds

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


@pytest.mark.parametrize("stream", [0, 1])
@pytest.mark.parametrize("src_kind", _kinds(), ids=str)
@pytest.mark.parametrize("dst_kind", _kinds(), ids=str)
def test_pairs_with_both_stores(stream, src_kind, dst_kind, monkeypatch):
    monkeypatch.setenv("RL_STREAM_STORES", str(stream))
    _check(W.CELL, src_kind, dst_kind, 20_011, seed=7, narrow=dst_kind[0] != "aos")


@pytest.mark.parametrize("stream", [0, 1])
def test_jagged_with_both_stores(stream, monkeypatch):
    monkeypatch.setenv("RL_STREAM_STORES", str(stream))
    _check(W.CLUSTER, ("aos", 0), ("soa", 0), 9_001, seed=13, mean_len=6)
    _check(W.CLUSTER, ("aos", 0), ("aosoa", 16), 9_001, seed=14, mean_len=6)


@pytest.mark.parametrize("stream", [0, 1])
def test_batch_with_both_stores(stream, monkeypatch):
    monkeypatch.setenv("RL_BATCH_STREAM", str(stream))
    monkeypatch.setenv("RL_BATCH_FANOUT", "128")
    b = _run(_shared_source_items("aos", 10_007), 128)
    assert b.info().stream_stores == stream
