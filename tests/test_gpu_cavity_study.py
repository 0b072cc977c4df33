"""The lid-driven cavity study runner (paper_2411_13992_amd.cavity) end to end
on a coarse cavity: the run stays finite and in range, the lid drags the fluid
below it along (u > 0 under the lid, a return flow u < 0 lower on the centre
line), and the two formulations give nearby profiles."""
import json

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def test_cavity_runner(tmp_path):
    from paper_2411_13992_amd import cavity
    out = tmp_path / "cavity.json"
    res = cavity.main(["--n", "30", "40", "--t-end", "2", "--json", str(out)])
    runs = res["runs"]
    assert len(runs) == 4 and all(r["flags"] == 0 for r in runs)
    for r in runs:
        u = np.asarray(r["u"])
        assert np.all(np.isfinite(u)) and np.all(np.isfinite(r["v"]))
        assert u[-1] > 0.1            # just under the lid
        assert u.min() < -0.01        # return flow
        assert np.abs(u).max() < 1.0 and np.abs(r["v"]).max() < 1.0
    assert set(res["convergence"]) == {"limited", "scaled"}
    for f in res["formulations"]:
        assert f["rms_u"] < 0.1 and f["rms_v"] < 0.1
    assert json.loads(out.read_text())["runs"][0]["n"] == 30
