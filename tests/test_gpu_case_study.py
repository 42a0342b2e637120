"""The case study's pipelines end to end on the device (Sec. VIII): sensor
records filled on the host, transferred into device SoA columns with the
conversion, energy computed (stand-in); particles reconstructed (stand-in)
and transferred back into the original record layout with their member
pool.  Parity claims cover the layout steps: the device columns after the
transfer and the host records after the transfer back are compared byte
for byte with the oracle's conversions of the same bytes.  The stand-in
arithmetic is compared with numpy within float32 rounding only."""
import numpy as np
import pytest

import oracle
import paper_2511_04853_amd as P
import workloads as W
import workloads.case_study as C

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    P.lib()


def test_sensor_and_particle_pipelines_layout_steps():
    side, npart = 96, 60
    v = C.sensor_grid(side, seed=7)
    stream = torch.cuda.current_stream()
    runs, host, cols, typed = C.sensor_pipeline(P, torch, side, v, stream, reps=1)
    S = oracle.Schema(W.SENSOR)
    aos, soa = oracle.make_layout(S, "aos"), oracle.make_layout(S, "soa")
    # the host fill: the records the oracle packs from the same values
    want_rec = oracle.pack(S, v, aos)[0]
    assert np.array_equal(host.numpy(), want_rec)
    # the transfer + conversion: every column but the energy (overwritten
    # by the stand-in) as the oracle converts the records
    st, want, _ = oracle.convert(aos, [want_rec], soa, v.n)
    assert st == 0
    got = [c.cpu().numpy() for c in cols]
    for k, (g, w) in enumerate(zip(got, want)):
        if k != 2:
            assert np.array_equal(g, w), f"sensor column {k}"
    e = got[2].view(np.float32)
    assert np.allclose(e, C.sensor_energy_numpy(v), rtol=1e-6, atol=1e-4)

    seeds = C.seed_sensors(side, npart, seed=8)
    pruns, dbufs, hbufs = C.particle_pipeline(P, torch, side, seeds, typed, stream, reps=1)
    tot = pruns[0]["members"]
    PS = oracle.Schema(W.PARTICLE)
    psoa, paos = oracle.make_layout(PS, "soa"), oracle.make_layout(PS, "aos")
    dev = [b.cpu().numpy() for b in dbufs]
    dev[-1] = dev[-1][:8 * tot]
    st, want, _ = oracle.convert(psoa, dev, paos, npart, [tot], [25 * npart])
    assert st == 0
    rec_bytes = npart * paos.stride
    assert np.array_equal(hbufs[0].numpy()[:rec_bytes], want[0][:rec_bytes]), "particle records"
    assert np.array_equal(hbufs[1].numpy()[:8 * tot], want[1][:8 * tot]), "particle member pool"
    # stand-in reconstruction against numpy: energy sums and member lists
    members = np.frombuffer(hbufs[1].numpy()[:8 * tot].tobytes(), np.int64)
    offs = np.concatenate([[0], np.cumsum(dev[len(dev) - 2].view(np.int32)[1:] - dev[len(dev) - 2].view(np.int32)[:-1])])
    en = e
    for k, s0 in enumerate(seeds):
        x0, y0 = s0 % side, s0 // side
        nb = [(y * side + x) for y in range(y0 - 2, y0 + 3) for x in range(x0 - 2, x0 + 3)
              if 0 <= x < side and 0 <= y < side]
        assert list(members[offs[k]:offs[k + 1]]) == nb
        assert np.isclose(dev[0].view(np.float32)[k], en[nb].sum(), rtol=1e-5)
