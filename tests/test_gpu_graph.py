"""A build captured once as a HIP graph and replayed: every replay equals the
eager build of the same reads, with eager work and synchronisations between the
replays, and new reads of the same shape copied into the captured buffers give
their own tables."""

import numpy as np
import pytest

import oracle
from paper_1003_1940_amd import synth
from .gpu_util import FIELDS, say

pytestmark = pytest.mark.gpu


def _same(a, b, label):
    for f in FIELDS:
        if a[f] is None or b[f] is None:
            continue
        assert np.array_equal(a[f], b[f]), f"{label}: column {f} differs"


def _reads(seed, n_reads=3000, genome=20_000, err=0.01):
    rng = np.random.default_rng(seed)
    g = synth.random_genome(rng, genome)
    return synth.sample_reads(rng, g, n_reads, 100, err)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible: the GPU tests need the MI355X")


@pytest.mark.parametrize("k", [31, 63])
def test_plain_graph_replays(k):
    import torch
    from paper_1003_1940_amd import api
    a, b = _reads(1), _reads(2)
    assert a.n_bases == b.n_bases and a.n_reads == b.n_reads
    say(f"[gpu-graph] plain k={k}: capture")
    packed, offs, nb = api.upload(a.bases, a.offsets)
    n_k = a.kmer_count(k)
    cap = api.CapturedBuild(packed, nb, offs, k, n_k)
    eager_a = api.build(a.bases, a.offsets, k).to_numpy()
    eager_b = api.build(b.bases, b.offsets, k).to_numpy()
    for rep in range(3):
        say(f"[gpu-graph] plain k={k}: replay {rep} (reads a)")
        cap.replay()
        torch.cuda.synchronize()
        g = cap.graph_result()
        assert g.status == 0
        _same(g.to_numpy(), eager_a, f"replay {rep}")
        # eager work between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int64)
        assert int(x.sum().item()) == (1 << 20) * ((1 << 20) - 1) // 2
    # other reads of the same shape through the same graph
    pb, ob, _ = api.upload(b.bases, b.offsets)
    cap.packed.copy_(pb)
    cap.offsets.copy_(ob)
    say(f"[gpu-graph] plain k={k}: replay with reads b")
    cap.replay()
    torch.cuda.synchronize()
    g = cap.graph_result()
    _same(g.to_numpy(), eager_b, "reads b")
    ref = oracle.build_graph(b.bases, b.offsets, k)
    assert g.n_nodes == len(ref.node_count) and g.n_edges == len(ref.edge_mult)


def test_batched_graph_replays():
    import torch
    from paper_1003_1940_amd import api
    sets = synth.batched_sets(n_sets=8, scale=0.003)
    bases = np.concatenate([s.bases for s in sets])
    lens = np.concatenate([np.diff(s.offsets.astype(np.int64)) for s in sets])
    offsets = np.zeros(len(lens) + 1, np.uint64)
    np.cumsum(lens, out=offsets[1:])
    sro = np.zeros(len(sets) + 1, np.uint64)
    np.cumsum([s.n_reads for s in sets], out=sro[1:])
    n_k = int(np.maximum(lens - 31 + 1, 0).sum())
    packed, offs, nb = api.upload(bases, offsets)
    sets_d = torch.from_numpy(sro.view(np.int64).copy()).cuda()
    say("[gpu-graph] batched: capture")
    cap = api.CapturedBuild(packed, nb, offs, 31, n_k, set_offsets=sets_d)
    eager = api.build_batched(bases, offsets, sro, 31)
    e = eager.to_numpy()
    for rep in range(3):
        say(f"[gpu-graph] batched: replay {rep}")
        cap.replay()
        torch.cuda.synchronize()
        g = cap.graph_result()
        assert g.status == 0
        _same(g.to_numpy(), e, f"batched replay {rep}")
        assert torch.equal(g.node_set_offsets, eager.node_set_offsets)
        assert torch.equal(g.edge_set_offsets, eager.edge_set_offsets)
        y = torch.ones(1000, device="cuda").cumsum(0)
        assert float(y[-1].item()) == 1000.0


def test_autotune_settings_agree():
    """Every tuning candidate builds identical tables (the tuner checks this
    itself and raises otherwise); the endpoint candidates take that route on a
    high-coverage input, and the choice is one of the candidates."""
    from paper_1003_1940_amd import api, autotune
    rng = np.random.default_rng(77)
    g = synth.random_genome(rng, 20_000)
    rs = synth.sample_reads(rng, g, 4000, 100, 0.001)
    for k in (31, 63):
        say(f"[gpu-graph] autotune k={k}")
        r = autotune.tune(rs.bases, rs.offsets, k, reps=1)
        assert len(r.timings_ms) == (36 if k > 31 else 18)
        assert r.best in [s for s, _, _ in r.timings_ms]
        for s, _, took in r.timings_ms:
            assert took == (s["node_path"] == api.NODES_ENDPOINTS), s
    assert api.get_tuning() == {"node_path": api.NODES_AUTO, "endpoint_ratio": pytest.approx(0.6),
                                "local_variant": 2, "lds_digit_bias": 0, "in_tile": 1}
