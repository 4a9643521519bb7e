"""GPU tests of one batched forward pass over ciphertexts of several clients, each with its own
evaluation keys (ctl_forward_multi): every output equals the client's own forward pass of that
ciphertext alone, bit for bit, and one client's outputs are checked against the oracle with that
client's keys."""
import functools

import numpy as np
import pytest

import workloads as W
from oracle import CKKSOracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CLIENT_SEEDS = (101, 202, 303)


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@functools.lru_cache(maxsize=None)
def _setup(name, lazy):
    _need_gpu()
    import paper_2205_11935_amd as ctl
    w = W.WORKLOADS[name]
    c = ctl.Context.for_workload(w)
    o = CKKSOracle.for_workload(w)
    plan = o.plan([(l.n_in, l.n_out, l.t1) for l in w.layers], lazy=bool(lazy), qp=lazy == "qp")
    banks = [W.raw_plaintexts(61 + li, L.t, o.n, bound_bits=45, stream=li) for li, L in enumerate(plan.layers)]
    model = c.load_model_raw([(l.n_in, l.n_out, l.t1) for l in w.layers], banks, lazy=bool(lazy), qp=lazy == "qp")
    keys = [c.keygen(s, model.info.rotations, relin=True) for s in CLIENT_SEEDS]
    return ctl, w, c, o, plan, banks, model, keys


def _batch(c, o, keys, owners, seed):
    msgs = W.raw_plaintexts(seed, len(owners), o.n, bound_bits=40)
    dev = c.empty_ct(len(owners), o.nq)
    for i, who in enumerate(owners):
        c.encrypt(keys[who], msgs[i], seed * 1000 + i, out=dev[i])
    return dev, msgs


@pytest.mark.parametrize("name,lazy", [("mid", False), ("mid", "qp"), ("large", "qp")])
def test_mixed_clients_equal_each_alone(name, lazy):
    ctl, w, c, o, plan, banks, model, keys = _setup(name, lazy)
    owners = [0, 0, 1, 2, 0, 1, 1, 2]              # runs of 2, 1, 1, 1, 2, 1
    dev, _ = _batch(c, o, keys, owners, 71)
    got = ctl.to_numpy_u64(c.forward_multi(model, [keys[i] for i in owners], dev))
    assert got.shape == (len(owners), 2, plan.k_out, o.n)
    for b, who in enumerate(owners):
        alone = ctl.to_numpy_u64(c.forward(model, keys[who], dev[b:b + 1].contiguous()))[0]
        assert np.array_equal(got[b], alone), (b, who)
    # the same keys for every ciphertext reduce to ctl_forward
    same = ctl.to_numpy_u64(c.forward_multi(model, [keys[0]] * len(owners), dev))
    assert np.array_equal(same, ctl.to_numpy_u64(c.forward(model, keys[0], dev)))


@pytest.mark.parametrize("name,lazy", [("mid", False), ("mid", "qp"), ("large", "qp")])
def test_mixed_clients_against_oracle(name, lazy):
    """Client 1's ciphertexts, batched between client 0's and 2's, against the oracle run with
    client 1's key seed."""
    ctl, w, c, o, plan, banks, model, keys = _setup(name, lazy)
    owners = [0, 1, 2, 1]
    dev, msgs = _batch(c, o, keys, owners, 72)
    got = ctl.to_numpy_u64(c.forward_multi(model, [keys[i] for i in owners], dev))
    seed = CLIENT_SEEDS[1]
    s = o.keygen_secret(seed)
    pk = o.keygen_public(seed, s)
    okeys = o.keygen_rotations(seed, s, plan.rotations)
    rlk = o.keygen_relin(seed, s)
    banks_ntt = [o.bank_ntt(banks[li], L.k, ext=lazy == "qp") for li, L in enumerate(plan.layers)]
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=2) as ex:      # the C oracle releases the interpreter lock
        wants = list(ex.map(lambda b: o.forward(plan, o.encrypt(pk, msgs[b], 72 * 1000 + b), banks_ntt, okeys, rlk),
                            (1, 3)))
    for b, want in zip((1, 3), wants):
        assert np.array_equal(got[b], want), b


def test_missing_key_in_one_run_is_rejected():
    ctl, w, c, o, plan, banks, model, keys = _setup("mid", False)
    partial = c.keygen(404, model.info.rotations[:-1], relin=True)
    dev, _ = _batch(c, o, keys, [0, 0], 73)
    out = c.empty_ct(2, model.info.k_out)
    before = ctl.to_numpy_u64(out).copy()
    with pytest.raises(ctl.CtlError) as e:
        c.forward_multi(model, [keys[0], partial], dev, out=out)
    assert e.value.code == -5                      # CTL_EKEY
    assert np.array_equal(ctl.to_numpy_u64(out), before)
    with pytest.raises(ValueError):
        c.forward_multi(model, [keys[0]], dev)
