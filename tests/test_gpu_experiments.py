"""The convection-cell drivers end to end on a small cell: a short boiling
run records finite Nusselt series, FP64-summed mass conservation, the
heat-flux pdf, the rho-T histograms and the structure functions; the adjoint
driver's FP64 gradients agree with its own central differences."""
import json

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1111_0905_amd import experiments, lbm
    lbm.load_library()
    return experiments


def test_convection_driver(ex, tmp_path):
    out = tmp_path / "c.json"
    ex.main(["convection", "--n", "32", "--ra", "1e5", "--steps", "400", "--diag", "100",
             "--phase-every", "200", "--out", str(out)])
    d = json.loads(out.read_text())
    assert d["ok"] and len(d["t"]) == 4
    assert np.all(np.isfinite(d["nu_bot"])) and np.all(np.isfinite(d["nu_z"]))
    assert abs(d["mass_drift"][-1]) < 1e-7
    pdf = d["bulk_flux_pdf"]
    assert sum(pdf["counts"]) + pdf["out_of_range"] == pdf["samples"] == 2 * 32 * 32 * 16
    for region in ("bottom", "bulk", "top"):
        c = np.asarray(d["rho_T_hist"][region]["counts"])
        assert c.shape == (150, 100)
    s = d["structure"]["vz"]
    assert len(s["S2"]) == 16 and np.all(np.asarray(s["S2"]) >= 0)
    assert len(d["phases_t"]) == 2


def test_adjoint_driver(ex, tmp_path):
    out = tmp_path / "a.json"
    ex.main(["adjoint", "--n", "16", "--ra", "1e5", "--steps", "20", "--ckpt", "5",
             "--out", str(out)])
    d = json.loads(out.read_text())
    for k in ("dJ_dTd", "dJ_dG", "dJ_drho0_dir"):
        assert d[f"fp64_vs_fd_rel_{k}"] < 1e-4
