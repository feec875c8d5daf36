"""What the trained network gains over the method without it: trained on the
GPU by the library's own kernels on a small set of random rooms, the learned
estimator's RT60 from a 1,024-ray trace is compared with the plain method's
RT60 from the same trace, both against an independent 65,536-ray reference."""
import numpy as np
import pytest

import paper_1803_00430_amd as P
import rpr_scenes as R
from paper_1803_00430_amd import learn as L

pytestmark = pytest.mark.gpu


def test_learned_estimator_beats_plain_at_1k_rays():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    train_rooms = [R.learn_room(10000 + i) for i in range(2048)]
    eval_rooms = [R.learn_room(200000 + i) for i in range(256)]
    tr_sc, ev_sc = L.make_scenes(train_rooms), L.make_scenes(eval_rooms)
    data = L.make_dataset(tr_sc, train_rooms, n_target=65536, inputs_per_room=4, chunk=1024)
    ev = L.make_dataset(ev_sc, eval_rooms, n_target=65536, chunk=1024)
    ref = L.trace_rooms(ev_sc, eval_rooms, n_rays=65536, seed_offset=L.SEED_REFERENCE, chunk=1024,
                        **L.CONVERGED)["params"]
    # the plain method on the very rays the network sees (1k rays, at the
    # estimator's own 1 ms bins and at the network's 10 ms bins)
    plain_1ms = L.trace_rooms(ev_sc, eval_rooms, n_rays=1024, seed_offset=L.SEED_INPUT, chunk=1024,
                              **L.CONVERGED)["params"]
    plain_10ms = L.trace_rooms(ev_sc, eval_rooms, n_rays=1024, seed_offset=L.SEED_INPUT, chunk=1024,
                               **L.INPUT)["params"]
    e_plain = min(L.rt60_error_summary(L.rt60_error(plain_1ms, ref, 4))["mean"],
                  L.rt60_error_summary(L.rt60_error(plain_10ms, ref, 4))["mean"])
    model = P.Model(P.LEARN_DIMS_TOWER, max_batch=256, seed=1)  # the default two-tower network
    model.set_tower(P.LEARN_DIMS_TOWER[0] - P.STAT_FEATURES, P.LEARN_TOWER)
    losses = L.train(model, data, epochs=12, lr=3e-4, weight_decay=1e-2, batch=128)
    assert losses[-1] < losses[0]
    prm, sig, unc = L.predict(model, ev["features"], ev["e_in"], 4, 1e9)
    e_learned = L.rt60_error_summary(L.rt60_error(prm, ref, 4))["mean"]
    print(f"RT60 error at 1k rays: plain {e_plain:.4f}, learned {e_learned:.4f}")
    assert e_learned < 0.5 * e_plain, (e_learned, e_plain)
    model.close()
