"""More GPU parity: random schemas over every layout pair, the benchmark's
own step (four conversions of the 190,000-object cell collection as one
autotuned batch), and a 2^24-object conversion compared in full."""
import ctypes

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import oracle
import paper_2511_04853_amd as P
import workloads as W
from tests import rlhelp as H
from tests.test_oracle_pins import schemas

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


KINDS = [("aos", 0), ("soa", 0), ("aosoa", 1), ("aosoa", 8), ("aosoa", 48)]


@settings(max_examples=40, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow, HealthCheck.function_scoped_fixture])
@given(decl=schemas(), si=st.integers(0, 4), di=st.integers(0, 4), n=st.sampled_from([1, 7, 100, 1001]))
def test_random_schemas_every_pair(decl, si, di, n):
    src_k, dst_k = KINDS[si], KINDS[di]
    if decl.offset_types and src_k[0] == "aos" and dst_k[0] == "aos":
        return   # not supported for jagged schemas
    sp = H.SchemaPair(decl)
    v = W.generic_values(decl, n, seed=n + 31 * si + 7 * di, mean_len=2.5)
    src, dst = sp.layout(*src_k), sp.layout(*dst_k)
    tot = H.totals(v)
    sbytes = oracle.pack(sp.orc, v, src.orc, pool_order=True)
    src_mem = ([len(sbytes[1 + g]) // src.orc.member_stride[g] for g in range(sp.orc.n_groups)]
               if src.kind == "aos" else tot)
    st_, want, _ = H.oracle_convert(src, sbytes, dst, n, src_mem, tot)
    assert st_ == 0
    rc, rs, got = H.run_lib_convert(src, sbytes, dst, n, src_mem, tot)
    assert rc == 0 and rs == 0, P.rl_last_error()
    H.assert_same_bytes(got, want, f"{src_k}->{dst_k} n={n}")


def test_benchmark_step_configuration(tmp_path):
    """The step bench.py times: AoS -> SoA and AoSoA 32/64/128 of 190,000
    cells (energy_d narrowed), one autotuned batch, against the oracle."""
    from tests.test_gpu_batch import Batch
    sp = H.SchemaPair(W.CELL)
    v = W.cell_values()
    aos = sp.layout("aos")
    narrow = H.narrowed_storage(W.CELL)
    dsts = [sp.layout("soa", storage=narrow)] + [sp.layout("aosoa", w, storage=narrow) for w in (32, 64, 128)]
    sbytes = oracle.pack(sp.orc, v, aos.orc)
    dsrc = H.to_device(sbytes)
    b = Batch(autotune=1, cache=str(tmp_path / "tune.json"))
    outs = []
    sv = P.View(aos.lib, v.n, dsrc)
    for d in dsts:
        dd = H.alloc_device(d.lib.buffer_bytes(v.n))
        outs.append(dd)
        b.add(sv, P.View(d.lib, v.n, dd), v.n)
    b.finalize()
    for rep in range(2):
        for dd in outs:
            for t in dd:
                t.fill_(H.SENTINEL)
        b.launch()
        assert P.sync() == 0, P.rl_last_error()
        for d, dd in zip(dsts, outs):
            st_, want, _ = H.oracle_convert(aos, sbytes, d, v.n, [], [])
            H.assert_same_bytes(H.to_numpy(dd), want, f"step {d.kind}{d.width}")


@pytest.mark.timeout(300)
def test_large_collection_in_full():
    """2^24 cells AoS -> SoA (narrowed): every byte against the oracle."""
    n = 1 << 24
    sp = H.SchemaPair(W.CELL)
    v = W.cell_values(n, seed=77)
    aos, soa = sp.layout("aos"), sp.layout("soa", storage=H.narrowed_storage(W.CELL))
    sbytes = oracle.pack(sp.orc, v, aos.orc)
    st_, want, _ = H.oracle_convert(aos, sbytes, soa, n, [], [])
    assert st_ == 0
    rc, rs, got = H.run_lib_convert(aos, sbytes, soa, n, [], [])
    assert rc == 0 and rs == 0
    H.assert_same_bytes(got, want, "2^24 cells")
