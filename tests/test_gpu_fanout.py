"""GPU parity of the batch fan-out path: dense steps that read the same
source tiles (one source converted into several layouts) share one
work-group per source tile, the tile brought into LDS once and each thread
group storing its own destination.  Forced on at both thread-group sizes,
several tile sizes and small grids (every work-group walks several groups
and tiles), with groups of four, a lone remainder step, steps that cannot
join (records, jagged scans) and unrelated items in the same batch; every
destination against the oracle byte for byte."""
import pytest

import paper_2511_04853_amd as P
from tests import rlhelp as H
from tests.test_gpu_batch import DECLS, Batch, Item, SharedSourceItem, _check_against_oracle, _small_specs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def _shared_source_items(src, n, schemas_used=("plain8", "cell", "cluster"), others=6):
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    items = []
    for sname in schemas_used:
        base = Item(schemas, dict(schema=sname, n=n, src=src, dst="soa" if src != "soa" else "aos"))
        items.append(base)
        narrow = H.narrowed_storage(DECLS[sname]) if sname == "cell" else None
        for dk, w in (("soa", None), ("aosoa", 32), ("aosoa", 3), ("aosoa", 128), ("aosoa", 64), ("aos", None)):
            if dk == src:
                continue
            items.append(SharedSourceItem(base, dk, narrow=None if dk == "aos" else narrow, width=w))
    if others:
        items += [Item(schemas, s) for s in _small_specs(others, seed=91)]
    return items


def _run(items, per=None):
    b = Batch()
    for it in items:
        b.add(it.sv, it.dv, it.n)
    b.finalize()
    info = b.info()
    if per:
        # every source with two or more direct destinations forms groups
        assert info.fanout_threads == per and info.fanout_groups > 0 and info.fanout_steps >= 2 * info.fanout_groups
    else:
        assert info.fanout_groups == 0 and info.fanout_threads == 0
    for mode in ("graph", "loop"):
        for it in items:
            for t in it.ddst:
                if t is not None:
                    t.fill_(H.SENTINEL)
        (b.launch if mode == "graph" else b.loop)()
        assert P.sync() == 0, P.rl_last_error()
        _check_against_oracle(items, b)
    return b


@pytest.mark.parametrize("src", ["aos", "soa", "aosoa"])
@pytest.mark.parametrize("per", [64, 128])
def test_fanout_one_source_into_several_layouts(src, per, monkeypatch):
    monkeypatch.setenv("RL_BATCH_FANOUT", str(per))
    _run(_shared_source_items(src, 30_001), per)


@pytest.mark.parametrize("pipe", [0, 1], ids=["one_slot", "double_buffered"])
@pytest.mark.parametrize("tile,grid", [(64, 3), (128, 0), (512, 11), (1024, 1)])
def test_fanout_tiles_and_grids(tile, grid, pipe, monkeypatch):
    """Small grids: work-groups step through the tiles of several groups
    (the group is found by walking the group ranges); double-buffered, the
    next tile's DMA overlaps the current tile's stores."""
    monkeypatch.setenv("RL_BATCH_FANOUT", "64")
    monkeypatch.setenv("RL_BATCH_TILE", str(tile))
    monkeypatch.setenv("RL_BATCH_PIPE", str(pipe))
    if grid:
        monkeypatch.setenv("RL_BATCH_GRID", str(grid))
    b = _run(_shared_source_items("aos", 5_003), 64)
    # two slots of 1,024 cell records (33 KB each) exceed 64 KB: one slot
    assert b.info().double_buffered == (pipe if tile <= 512 else 0)


@pytest.mark.parametrize("src", ["soa", "aosoa"])
def test_fanout_double_buffered_other_sources(src, monkeypatch):
    monkeypatch.setenv("RL_BATCH_FANOUT", "128")
    monkeypatch.setenv("RL_BATCH_PIPE", "1")
    monkeypatch.setenv("RL_BATCH_GRID", "5")
    _run(_shared_source_items(src, 20_011), 128)


def test_fanout_partial_and_single_tiles(monkeypatch):
    """Sources of one object, of less than a tile and of a tile plus one."""
    monkeypatch.setenv("RL_BATCH_FANOUT", "128")
    monkeypatch.setenv("RL_BATCH_TILE", "256")
    for n in (1, 200, 257):
        _run(_shared_source_items("aos", n), 128)


@pytest.mark.parametrize("pipe", [0, 1], ids=["one_slot", "double_buffered"])
@pytest.mark.parametrize("per", [64, 128])
def test_fanout_groups_alone(per, pipe, monkeypatch):
    """A batch whose dense steps all sit in fan-out groups (no other dense
    tile, no gather): one source converted into four direct layouts."""
    monkeypatch.setenv("RL_BATCH_FANOUT", str(per))
    monkeypatch.setenv("RL_BATCH_PIPE", str(pipe))
    if pipe:
        monkeypatch.setenv("RL_BATCH_GRID", "64")
    schemas = {k: H.SchemaPair(d) for k, d in DECLS.items()}
    base = Item(schemas, dict(schema="cell", n=40_009, src="aos", dst="soa"))
    narrow = H.narrowed_storage(DECLS["cell"])
    base = SharedSourceItem(base, "soa", narrow=narrow)
    items = [base] + [SharedSourceItem(base, "aosoa", narrow=narrow, width=w) for w in (32, 64, 128)]
    b = _run(items, per)
    info = b.info()
    assert info.fanout_groups == 1 and info.fanout_steps == 4 == info.dense_steps


def test_fanout_off_by_default_without_tuning(monkeypatch):
    monkeypatch.delenv("RL_BATCH_FANOUT", raising=False)
    _run(_shared_source_items("aos", 3_001, others=0))
