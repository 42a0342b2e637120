"""GPU parity of the double-buffered dense pipeline (two tile slots per
work-group; a tile's source DMA issued before the previous tile's
transform, waited for with a partial vector-memory counter wait), forced on
with small grids so that every work-group converts tens of tiles: every
layout pair, narrowing, partial last tiles, destination images (records),
the fused jagged scan, records built from offsets columns, and a batch,
against the oracle byte for byte."""
import pytest

import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H
from tests.test_gpu_batch import DECLS, Batch, Item, _check_against_oracle, _small_specs
from tests.test_gpu_parity import _check, _kinds

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


@pytest.fixture
def pipelined(monkeypatch):
    monkeypatch.setenv("RL_PIPELINE", "1")
    monkeypatch.setenv("RL_GRID_BLOCKS", "5")


@pytest.mark.parametrize("decl", [W.PLAIN8, W.CELL, W.SENSOR], ids=lambda d: d.name)
@pytest.mark.parametrize("src_kind", _kinds(), ids=str)
@pytest.mark.parametrize("dst_kind", _kinds(), ids=str)
def test_every_pair_double_buffered(decl, src_kind, dst_kind, pipelined):
    _check(decl, src_kind, dst_kind, 30_011, seed=3, narrow=decl is W.CELL and dst_kind[0] != "aos")


@pytest.mark.parametrize("tile,threads", [(64, 64), (256, 128), (512, 256)])
def test_tile_shapes_double_buffered(tile, threads, pipelined, monkeypatch):
    monkeypatch.setenv("RL_TILE_OBJECTS", str(tile))
    monkeypatch.setenv("RL_BLOCK_THREADS", str(threads))
    _check(W.CELL, ("aos", 0), ("soa", 0), 50_001, seed=5, narrow=True)
    _check(W.CELL, ("aos", 0), ("aosoa", 128), 50_001, seed=5, narrow=True)
    _check(W.SENSOR, ("soa", 0), ("aos", 0), 50_001, seed=5)


def test_jagged_scan_and_offsets_records_double_buffered(pipelined, monkeypatch):
    """The multi-kernel jagged path: records with a fused per-tile scan,
    and records rebuilt from an offsets column (offsets staged with each
    tile), both double-buffered."""
    monkeypatch.setenv("RL_JAGGED_FUSED", "0")
    for pair in [(("aos", 0), ("soa", 0)), (("soa", 0), ("aos", 0)), (("aosoa", 16), ("aos", 0))]:
        _check(W.CLUSTER, pair[0], pair[1], 9_001, seed=11, mean_len=6)
        _check(W.PARTICLE, pair[0], pair[1], 9_001, seed=12, mean_len=3)


def test_long_conversion_single_slot_by_default():
    """A long conversion (16,384 tiles and more) on the default plan, which
    no longer double-buffers it, against the oracle."""
    _check(W.PLAIN8, ("aos", 0), ("soa", 0), 16384 * 512 + 77, seed=2)


def test_batch_double_buffered(monkeypatch):
    monkeypatch.setenv("RL_BATCH_PIPE", "1")
    monkeypatch.setenv("RL_BATCH_GRID", "7")
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    items = [Item(schemas, s, auto_width=False) for s in _small_specs()]
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    b.launch()
    assert P.sync() == 0, P.rl_last_error()
    _check_against_oracle(items, b)
    for it in items:
        for t in it.ddst:
            if t is not None:
                t.fill_(H.SENTINEL)
    b.launch()
    assert P.sync() == 0
    _check_against_oracle(items, b)
