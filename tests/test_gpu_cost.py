"""Cost model on the device: calibration (the one-time benchmark of Sec.
III-C), predictions of whole runs against their measured times, and the mode
SV_FUSE_AUTO picks, in sv_run and in the server."""
import time

import numpy as np
import pytest

import workloads as W
from test_gpu_serving import _check_vs_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def model(ctx, S):
    m = S.CostModel.calibrate(ctx, "c128", 8, 22)
    lo, hi, tab = m.table()
    assert (lo, hi) == (8, 22) and np.all(tab > 0)
    yield m
    ctx.set_cost_model(None)


def _measure(S, st, arr, fk):
    import torch

    st.reset(0)
    st.run(arr, fuse_k=fk)          # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st.reset(0)
    st.run(arr, fuse_k=fk)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


@pytest.mark.parametrize("name", ["brickwork", "qft", "random"])
def test_predictions_track_measured_runs(ctx, S, model, name):
    n = 20
    ops = {"brickwork": W.brickwork(n, 20, seed=3), "qft": W.qft(n),
           "random": W.random_circuit(n, 400, seed=4)}[name]
    arr = S.ops_to_numpy(ops)
    with S.State(ctx, n, "c128") as st:
        meas = {fk: _measure(S, st, arr, fk) for fk in (0, 5, -1)}
    pred = {fk: model.predict(ops, n, fk, 0) for fk in (0, 5, -1)}
    for fk in meas:
        # a reset (one full sweep) is inside the measured time
        ratio = pred[fk] / max(meas[fk] - model.coefficient("gate_full", n), 1e-6)
        assert 0.5 <= ratio <= 2.0, (name, fk, pred[fk], meas[fk])
    # the mode SV_FUSE_AUTO would pick is within 30 % of the fastest measured one
    pick = min(pred, key=pred.get)
    assert meas[pick] <= 1.3 * min(meas.values()), (name, pred, meas)


def test_auto_mode_in_run_and_server(ctx, S, O, model):
    ctx.set_cost_model(model)
    n = 10
    ops = W.random_circuit(n, 150, seed=9)
    with S.State(ctx, n, "c128") as st:
        st.run(ops, fuse_k=S.SV_FUSE_AUTO)
        got = st.copy_out()
    assert np.max(np.abs(got - O.run(ops, n))) <= 1e-12
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(12):
        nq = int(rng.integers(14, 19))
        reqs.append({"n": nq, "ops": W.serving_circuit(nq, int(rng.integers(5, 20)), rng), "shots": 300,
                     "seed": 1000 + i, "terms": [(0, 3, 1.0)], "dtype": "c128", "fuse_k": S.SV_FUSE_AUTO})
    with S.Server(ctx) as srv:
        ids = [srv.submit(r["n"], r["ops"], shots=r["shots"], seed=r["seed"], terms=r["terms"],
                          dtype=r["dtype"], fuse_k=r["fuse_k"]) for r in reqs]
        res = [srv.wait(i, 60000) for i in ids]
    for r, x in zip(reqs, res):
        _check_vs_oracle(O, r, x)
