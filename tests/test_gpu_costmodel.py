"""The launch-configuration cost model trained by the library's own GPU
kernels on the committed dataset of labelled random chains (features and
the 20 configurations' measured times, labelled by costmodel.py), and
evaluated on the held-out chains: the model's choice must stay within 10%
of the autotuned best in geometric mean, and beat the library's default
configuration."""
import os

import pytest

from paper_2508_07071_amd import costmodel as cm

pytestmark = pytest.mark.gpu

DATASET = os.path.join(os.path.dirname(cm.__file__), "data", "costmodel_dataset.npz")


@pytest.mark.skipif(not os.path.exists(DATASET), reason="labelled dataset not present")
def test_model_choice_on_held_out_chains():
    print("[case] cost model on the labelled dataset", flush=True)
    import paper_2508_07071_amd as fk
    data = cm.load_shards([DATASET])
    assert data["features"].shape == (cm.N_TRAIN + cm.N_TEST, fk.FK_MODEL_FEATURES)
    model, rep = cm.fit(data, epochs=100)
    try:
        assert rep["loss_last"] < rep["loss_first"]
        assert rep["model"]["geomean"] >= 0.90, rep
        assert rep["model"]["geomean"] > rep["default"]["geomean"], rep
    finally:
        fk.fk_model_destroy(model)
