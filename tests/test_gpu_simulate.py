"""The simulation driver runs every force mode end to end on a small load:
a few KDK steps from a = 0.02, axial momentum and force-error checks against
the FP64 GPU reference.  Bars per mode: the force error of the mode at the
last check (exact |n| <= 8: round-off; learned: network error; table and
complete: interpolation error; tree: opening-angle error) and the axial
momentum (conserved pair by pair except by the tree)."""
import json

import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sim():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20787_amd import simulate
    return simulate


# bars on the median and the largest force error of the last check
@pytest.mark.parametrize("mode,med,err,pz", [("exact", 1e-6, 2e-5, 1e-7), ("learned", 1e-5, 1e-4, 1e-7),
                                             ("table", 1e-4, 2e-3, 1e-7), ("complete", 1e-4, 2e-3, 1e-7),
                                             ("tree", 2e-2, 2.0, 1e-2)])
def test_driver_runs_each_mode(sim, capsys, mode, med, err, pz):
    rc = sim.main(["--N", "4096", "--steps", "4", "--mode", mode, "--check-every", "4",
                   "--check-targets", "256", "--a1", "0.05"])
    assert rc == 0
    out = capsys.readouterr().out.strip().splitlines()
    summary = json.loads(out[-1])
    assert summary["mode"] == mode and summary["steps"] == 4
    last = summary["checks"][-1]
    print(mode, last, summary["max_pz_ratio"])
    assert last["median_rel_err"] <= med
    assert last["max_rel_err"] <= err
    assert summary["max_pz_ratio"] <= pz


@pytest.mark.parametrize("argv", [["--path", "exact", "--targets", "1000", "--potential"],
                                  ["--path", "learned", "--targets", "4096"],
                                  ["--path", "table", "--order", "2"],
                                  ["--path", "table", "--order", "1", "--explicit-targets"],
                                  ["--path", "tree", "--quadrupole"]])
def test_profiling_driver_runs_each_path(capsys, argv):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20787_amd import run_kernel
    run_kernel.main(argv + ["--N", "8192", "--reps", "2"])
    row = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert row["path"] == argv[1] and row["N"] == 8192 and len(row["ms"]) == 2
    assert all(ms > 0 for ms in row["ms"])


@pytest.mark.parametrize("argv,bar", [(["--path", "exact", "--pairwise", "--n-img", "1024"], 1e-5),
                                      (["--path", "learned", "--pairwise"], 1e-4)])
def test_profiling_driver_checks_against_the_f64_reference(capsys, argv, bar):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2602_20787_amd import run_kernel
    run_kernel.main(argv + ["--N", "4096", "--reps", "1", "--check-targets", "128"])
    row = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert row["err_vs_f64"]["targets"] == 128
    assert row["err_vs_f64"]["max"] <= bar


def test_stop_after_runs_a_prefix_of_the_schedule(sim, capsys):
    # the first 3 of 6 steps: the same step sizes and, with deterministic
    # forces and kicks, the same state as the full run at step 3
    base = ["--N", "4096", "--steps", "6", "--mode", "exact", "--check-every", "3",
            "--check-targets", "256", "--a1", "0.05"]
    assert sim.main(base) == 0
    full = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert sim.main(base + ["--stop-after", "3"]) == 0
    part = json.loads(capsys.readouterr().out.strip().splitlines()[-1])
    assert part["steps_run"] == 3 and full["steps_run"] == 6
    assert part["a_reached"] == pytest.approx(full["checks"][1]["a"], rel=1e-15)
    assert part["checks"][-1]["step"] == 3
    assert part["checks"][-1]["max_rel_err"] == full["checks"][1]["max_rel_err"]
    assert part["checks"][-1]["median_rel_err"] == full["checks"][1]["median_rel_err"]
