"""GPU parity of batched channels (replicas of different size, particles per
cell, Knudsen number, force and seed stepped together).

Every replica must evolve exactly as the same channel alone: against the
oracle (one independent run per replica) cell starts and counters agree
exactly and FP64 particle values within 1e-12 relative (the single-channel
bar); against a one-channel GPU context of the same parameters, bit for bit.
The tiling (tile shapes per replica, chosen by particles per tile or by the
autotuner) must not change the particles, cell starts or counters; the
sampled moment sums add the same terms in an order that follows the tile
shape, so across tilings they agree to rounding.
"""
import numpy as np
import pytest
import torch

import inputs
from oracle import oracle as O

pytestmark = pytest.mark.gpu


def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1512_08042_amd import dsmc as D
    from paper_1512_08042_amd.config import ChannelConfig

    return D, ChannelConfig


REPS = [
    dict(nx=1, ny=40, ppc=60, kn=0.05, mach=0.1, seed=11),
    dict(nx=3, ny=7, ppc=25, kn=0.3, mach=0.0, seed=12),
    dict(nx=2, ny=13, ppc=9, kn=0.5, mach=0.2, seed=13),
    dict(nx=1, ny=33, ppc=120, kn=0.02, mach=0.1, seed=14),
    dict(nx=5, ny=5, ppc=40, kn=0.1, mach=0.1, seed=15),
    dict(nx=1, ny=64, ppc=7, kn=1.0, mach=0.05, seed=16),
]


def _oracle_of(rep, state32=False):
    r = rep
    ref = O.Sim(r["nx"], r["ny"], r["ppc"], r["kn"], dt=r["dt"], g=r["body_force_x"], seed=r["seed"],
                capacity=r["nx"] * r["ny"] * r["ppc"] + 64, state32=state32)
    ref.init_maxwell()
    return ref


def _check_replica(b, i, ref, tol=1e-12, what=""):
    cs = b.replica_cell_start(i).cpu().numpy()
    assert np.array_equal(cs, ref.cells()[0]), "replica %d cell_start %s" % (i, what)
    got = [t.cpu().numpy().astype(np.float64) for t in b.replica_particles(i)]
    for name, g, w in zip("x y vx vy vz".split(), got, ref.particles()):
        assert g.shape == w.shape, (i, name)
        assert np.allclose(g, w, rtol=tol, atol=tol), "replica %d %s %s" % (i, name, what)
    rc = ref.counters()
    assert tuple(int(v) for v in b.replica_counters()[i]) == (rc["ncoll"], rc["ncand"], rc["nwall"]), (i, what)


def test_batch_replicas_match_oracle_and_single_channels():
    D, ChannelConfig = _gpu()
    b = D.Batch(REPS)
    refs = [_oracle_of(r) for r in b.replicas]
    for _ in range(3):
        b.step(4, sample_every=1)
        for ref in refs:
            ref.step(4, sample_every=1)
    st = b.status()
    assert st["bits"] == 0 and st["n"] == sum(r["nx"] * r["ny"] * r["ppc"] for r in REPS)
    avg = b.sample_moments().cpu().numpy()
    for i, ref in enumerate(refs):
        _check_replica(b, i, ref, what="after 12 steps")
        c0, c1 = b.replica_cells(i)
        want = ref.averages()
        scale = np.abs(want).max(axis=1, keepdims=True) + 1.0
        assert np.all(np.abs(avg[:, c0:c1] - want) <= 1e-12 * scale), "replica %d moments" % i
    # the same replica alone, on the GPU: bit for bit
    for i in (0, 2, 4):
        r = b.replicas[i]
        ch = D.Channel(ChannelConfig(nx=r["nx"], ny=r["ny"], ppc=r["ppc"], kn=r["kn"], dt=r["dt"],
                                     body_force_x=r["body_force_x"], seed=r["seed"]))
        for _ in range(3):
            ch.step(4, sample_every=1)
        for g, w in zip(b.replica_particles(i), ch.particles()):
            assert torch.equal(g, w), "replica %d differs from its channel run alone" % i
        ch.close()
    b.close()


def test_tiling_and_autotuner_do_not_change_results():
    D, _ = _gpu()
    runs = []
    for ppt in (0, 50, 100, 800, "auto"):
        b = D.Batch(REPS)
        if ppt == "auto":
            tune = b.autotune(steps_per_trial=2, sample_every=1)  # 8 real steps
            assert tune["chosen"] in tune["particles_per_tile"] and len(tune["ms_per_step"]) == 4
            b.step(2, sample_every=1)
        else:
            b.set_tiling(ppt)
            b.step(4, sample_every=1)
            b.step(3, sample_every=1)
            b.step(3, sample_every=1)
        runs.append(([t.cpu().numpy().copy() for t in b.particles()], b.cell_start().cpu().numpy().copy(),
                     b.sample_moments().cpu().numpy(), b.replica_counters().copy()))
        b.close()
    for other in runs[1:]:
        for a, c in zip(runs[0][0], other[0]):
            assert np.array_equal(a, c)
        assert np.array_equal(runs[0][1], other[1]) and np.array_equal(runs[0][3], other[3])
        # the moment sums add the same terms in an order that follows the tile
        # shape (the lanes sharing a cell): equal to rounding
        scale = np.abs(runs[0][2]).max(axis=1, keepdims=True) + 1.0
        assert np.all(np.abs(runs[0][2] - other[2]) <= 1e-13 * scale)


def test_fp32_batch_matches_fp32_oracle():
    D, _ = _gpu()
    b = D.Batch(REPS[:4], state_bits=32)
    refs = [_oracle_of(r, state32=True) for r in b.replicas]
    b.step(6, sample_every=1)
    for ref in refs:
        ref.step(6, sample_every=1)
    for i, ref in enumerate(refs):
        _check_replica(b, i, ref, tol=2.0 * 2.0 ** -23, what="FP32 after 6 steps")
    b.close()


def test_batch_rejects_the_single_channel_mappings():
    D, _ = _gpu()
    from paper_1512_08042_amd._lib import ESTATE, DsmcError

    b = D.Batch(REPS[:2])
    b.step(1, sample_every=1)
    with pytest.raises(DsmcError) as e:
        b.map_to_lbm(9, 2)
    assert e.value.code == ESTATE
    b.close()


def test_256_uneven_replicas_sampled_against_the_oracle():
    # the batched workload: 256 replicas, ny in [32, 512], ppc in [20, 200],
    # Kn log-uniform in [0.01, 1], Ma 0.1, seeds 1000 + r; two steps, then the
    # smallest, a middle and the largest replica against the oracle
    D, _ = _gpu()
    reps = inputs.replica_params(3, 256)
    for r in reps:
        r["mach"] = 0.1
    b = D.Batch(reps)
    b.step(2, sample_every=1)
    st = b.status()
    npart = [r["ny"] * r["ppc"] for r in reps]
    assert st["bits"] == 0 and st["n"] == sum(npart)
    order = np.argsort(npart)
    for i in (int(order[0]), int(order[128]), int(order[-1])):
        ref = _oracle_of(b.replicas[i])
        ref.step(2, sample_every=1)
        _check_replica(b, i, ref, what="256-replica batch, replica %d" % i)
    b.close()


def test_step_graph_replays_match_eager_steps():
    # one dsmc_step(4 steps, sampling every step) captured into a HIP graph and
    # replayed three times, with eager work and synchronisation between the
    # replays; after every replay the state equals that of the same steps run
    # eagerly on a second context
    D, _ = _gpu()
    from paper_1512_08042_amd._lib import ESTATE, DsmcError

    s = torch.cuda.Stream()
    eager = D.Batch(REPS)
    graphed = D.Batch(REPS)
    torch.cuda.synchronize()
    graphed.graph_create(4, sample_every=1, stream=s)
    for rep in range(3):
        eager.step(4, sample_every=1)
        graphed.graph_launch(stream=s)
        s.synchronize()
        _ = eager.status()  # eager work between replays
        got = [t.cpu().numpy() for t in graphed.particles()]
        want = [t.cpu().numpy() for t in eager.particles()]
        for g, w in zip(got, want):
            assert np.array_equal(g, w), "replay %d" % rep
        assert np.array_equal(graphed.cell_start().cpu().numpy(), eager.cell_start().cpu().numpy())
        assert np.array_equal(graphed.sample_moments().cpu().numpy(), eager.sample_moments().cpu().numpy())
        assert np.array_equal(graphed.replica_counters(), eager.replica_counters())
        assert graphed.views().step == eager.views().step == 4 * (rep + 1)
    # an odd number of eager steps breaks the captured parity: refused
    graphed.step(1, sample_every=1)
    with pytest.raises(DsmcError) as e:
        graphed.graph_launch(stream=s)
    assert e.value.code == ESTATE
    torch.cuda.synchronize()
    eager.close()
    graphed.close()


def test_retiling_releases_the_step_graph():
    # a graph holds the tile shapes it was captured with: a re-tiling
    # releases it (a replay is refused, with the reason in the context's
    # message), and a graph captured after the re-tiling replays like eager
    # steps under the new tiling
    D, _ = _gpu()
    from paper_1512_08042_amd._lib import ESTATE, DsmcError

    s = torch.cuda.Stream()
    eager = D.Batch(REPS)
    graphed = D.Batch(REPS)
    torch.cuda.synchronize()
    graphed.graph_create(2, sample_every=1, stream=s)
    graphed.graph_launch(stream=s)
    eager.step(2, sample_every=1)
    graphed.set_tiling(100, stream=s)  # smaller tiles: two replicas change shape
    with pytest.raises(DsmcError) as e:
        graphed.graph_launch(stream=s)
    assert e.value.code == ESTATE
    assert "graph" in e.value.detail and "dsmc_graph_launch" in e.value.detail
    graphed.graph_create(2, sample_every=1, stream=s)
    for rep in range(2):
        graphed.graph_launch(stream=s)
        eager.step(2, sample_every=1)
        s.synchronize()
        for g, w in zip(graphed.particles(), eager.particles()):
            assert np.array_equal(g.cpu().numpy(), w.cpu().numpy()), "replay %d after re-tiling" % rep
        assert np.array_equal(graphed.cell_start().cpu().numpy(), eager.cell_start().cpu().numpy())
        assert np.array_equal(graphed.replica_counters(), eager.replica_counters())
    torch.cuda.synchronize()
    eager.close()
    graphed.close()


def test_last_error_names_the_call_and_the_reason():
    D, _ = _gpu()
    from paper_1512_08042_amd._lib import EINVAL, ESTATE, DsmcError

    b = D.Batch(REPS[:2])
    with pytest.raises(DsmcError) as e:
        b.step(-1)
    assert e.value.code == EINVAL
    assert e.value.detail.startswith("dsmc_step: nsteps") and "invalid argument" in e.value.detail
    with pytest.raises(DsmcError) as e:
        b.map_to_lbm(9, 2)
    assert e.value.code == ESTATE and "one channel only" in e.value.detail
    b.step(1)  # a successful call leaves the message of the last failure
    from paper_1512_08042_amd._lib import lib

    assert lib().dsmc_last_error(b._h).decode().startswith("map_dsmc_to_lbm:")
    b.close()
