"""The experiment tools (alpha sweep, convergence study, Reynolds sweep, eq. (14)
measurement) run end to end on short versions of their workloads and print
well-formed JSON records."""
import json

import pytest

from paper_2006_10487_amd import hlbm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hlbm.lib()


def records(capsys):
    out = capsys.readouterr().out
    return [json.loads(line) for line in out.splitlines() if line.startswith("{")]


def test_polar_tool(capsys):
    from paper_2006_10487_amd import polar
    assert polar.main(["--aoa", "0,4", "--steps", "200", "--ns", "512"]) == 0
    r = records(capsys)
    assert [x["aoa_deg"] for x in r] == [0.0, 4.0]
    for x in r:
        assert x["fp64"]["cd"] > 0 and x["cd_rel_err"] < 1e-3
    assert abs(r[0]["fp64"]["cl"]) < 1e-10 and abs(r[1]["fp64"]["cl"]) > 1e-6


def test_convergence_tool(capsys):
    from paper_2006_10487_amd import convergence
    assert convergence.main(["--chords", "48,64,96", "--passes", "0.2"]) == 0
    r = records(capsys)
    assert [x["chord"] for x in r[:3]] == [48, 64, 96]
    assert all(x["n_sub"] == 70 and x["cl_abs_max"] < 1e-8 for x in r[:3])
    assert "p" in r[3] and set(r[3]["err_pct"]) == {"48", "64", "96"}


def test_resweep_tool(capsys):
    from paper_2006_10487_amd import resweep
    assert resweep.main(["--re", "1000", "--passes", "0.02"]) == 0
    (x,) = records(capsys)
    assert x["n_sub"] == 14 and x["paper_cd_c1024"] == 0.119
    assert x["fp64"]["cd"] > 0 and x["cd_rel_err"] < 1e-3


def test_speedup_tool(capsys):
    from paper_2006_10487_amd import speedup
    assert speedup.main(["--workload", "naca_re1000_c128", "--steps", "4", "--warmup", "1"]) == 0
    (x,) = records(capsys)
    assert x["t_h_ms_per_base_step"] > 0 and x["t_eq_ms_per_base_step"] > 0
    m = x["model"]
    assert m["n"] == 53 and m["g"] > 1 and 0 < m["chi"] < 1
    ratio = x["t_h_ms_per_base_step"] / x["t_eq_ms_per_base_step"]   # both rounded to 1e-4 ms
    assert abs(x["G_measured"] - ratio) < 2e-3 * ratio
    assert x["equivalent_body"]["solid_nodes"] > 5000 and x["equivalent_body"]["bounce_back_nodes"] > 500
    assert x["t_eq_nobody_ms_per_base_step"] > 0


def test_speedup_accuracy_comparison(capsys):
    """Both schemes over the same physical time: the equivalent LBM takes twice the
    finest steps, and the impulsive start gives finite, positive mean drag for both."""
    from paper_2006_10487_amd import speedup
    assert speedup.main(["--workload", "naca_re100_c40", "--steps", "2", "--warmup", "1",
                         "--fp64", "--accuracy-steps", "400", "--aoa", "0"]) == 0
    (x,) = records(capsys)
    acc = x["accuracy"]
    assert acc["hybrid"]["finest_steps"] == 400 and acc["equivalent_lbm"]["finest_steps"] == 800
    for k in ("hybrid", "equivalent_lbm"):
        assert acc[k]["cd_mean"] > 0 and abs(acc[k]["cl_mean"]) < 1e-10


def test_wallprofile_tool(capsys):
    from paper_2006_10487_amd import wallprofile
    assert wallprofile.main(["--aoa", "8", "--steps", "200", "--ns", "512"]) == 0
    (x,) = records(capsys)
    assert x["steps_averaged"] == 100
    for side in ("upper", "lower"):
        s = x[side]
        assert len(s["cp"]) == len(s["cf"]) == len(s["x_stations"]) == 21
        assert s["x_stations"][0] == 0.0 and s["x_stations"][-1] == 1.0
    # stagnation on the lower side of the leading edge at positive incidence: the
    # suction peak is on the upper surface
    assert x["upper"]["cp_min"] < x["lower"]["cp_min"]
