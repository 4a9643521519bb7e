"""Autotuner: cache keys and the JSON cache on the CPU; on the GPU, tuning a batched forward pass
leaves every result bit-identical (the tuner checks each candidate) and settles on valid knobs."""
import json

import numpy as np
import pytest

from paper_2205_11935_amd import autotune


class FakeCtx:
    def __init__(self):
        self.k = {"mac_chunk": 16, "mac_cts": 8, "keyip_xcd": 1}

    def knob(self, name, value=None):
        if value is not None:
            self.k[name] = value
        return self.k[name]


def test_pick_keeps_entry_within_margin():
    # a candidate replaces the value on entry only when faster by more than the margin
    assert autotune.pick({128: 18.10, 0: 18.00, 64: 18.05}, 128, 0.01) == 128
    assert autotune.pick({128: 18.50, 0: 18.00}, 128, 0.01) == 0
    assert autotune.pick({4: 10.0, 8: 9.0}, 8, 0.01) == 8
    assert autotune.pick({4: 10.0, 8: 9.0}, 16, 0.01) == 8     # entry value not among the trials


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    k1 = autotune.cache_key("gfx950", 14, [3, 5, 7])
    k2 = autotune.cache_key("gfx950", 14, [3, 5, 11])
    assert k1 != k2 and k1.startswith("gfx950/N=2^14/")
    assert autotune.load(path, k1) is None
    autotune.save(path, k1, {"knobs": {"mac_chunk": 8, "mac_cts": 4, "keyip_xcd": 0}, "best_ms": 1.0})
    autotune.save(path, k2, {"knobs": {"mac_chunk": 12, "mac_cts": 8, "keyip_xcd": 1}, "best_ms": 2.0})
    assert autotune.load(path, k1) == {"mac_chunk": 8, "mac_cts": 4, "keyip_xcd": 0}
    ctx = FakeCtx()
    autotune.apply(ctx, autotune.load(path, k2))
    assert ctx.k == {"mac_chunk": 12, "mac_cts": 8, "keyip_xcd": 1}
    assert set(json.load(open(path))) == {k1, k2}


@pytest.mark.gpu
def test_tune_forward_pass_bit_identical():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_11935_amd as ctl
    import workloads as W
    w = W.MID
    c = ctl.Context.for_workload(w)
    m = c.load_model([(l.n_in, l.n_out, l.t1) for l in w.layers], W.weights(w), lazy=True, qp=True)
    keys = c.keygen(w.seed_keys, m.info.rotations, relin=True)
    ct = c.empty_ct(6, c.nq)
    for i in range(6):
        c.encrypt(keys, W.raw_plaintexts(90 + i, 1, c.n, 30)[0], 91 + i, out=ct[i])
    out = c.empty_ct(6, m.info.k_out)
    res = autotune.tune(c, lambda: c.forward(m, keys, ct, out=out), reps=2)
    assert set(res["knobs"]) == set(autotune.CANDIDATES)
    for name, v in res["knobs"].items():
        assert v in autotune.CANDIDATES[name] and c.knob(name) == v
    assert res["best_ms"] > 0
    with pytest.raises(ctl.CtlError):
        c.knob("mac_cts", 17)
    assert c.knob("mac_cts") == res["knobs"]["mac_cts"]
