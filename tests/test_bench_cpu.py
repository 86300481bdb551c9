"""Host logic of bench.py: the algorithmic byte model behind the roofline
figure, recounted array by array, and the one-GPU guard."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def recount(kind, n, fp):
    """Bytes per launch from the arrays each pass reads and writes (xfwd:
    residual evaluation, first and later CG iterations)."""
    v = n ** 3
    comp = fp * v                        # one real field component
    spectrum = 6 * n * n * (n // 2 + 1) * 2 * fp
    tangent = 2 * comp + v               # factors (a, b) and the phase byte
    if kind == "xfwd":
        return (6 * comp + spectrum,                 # read sigma, write the spectrum
                12 * comp + tangent + spectrum,      # read r and the tangent, write p and the spectrum
                30 * comp + tangent + spectrum)      # read r, p, x and the tangent, write p, x, spectrum
    if kind == "xinv":
        return spectrum + 12 * comp                  # read the spectrum and r (or sigma), write r
    return 2 * spectrum                              # y and z passes: the spectrum in and out


@pytest.mark.parametrize("n,fp", [(256, 4), (64, 8), (48, 4)])
def test_byte_model_matches_a_per_array_count(n, fp):
    assert bench.algorithmic_bytes("xfwd", n, fp, 0.8) == pytest.approx(recount("xfwd", n, fp), rel=1e-15)
    for kind in ("xinv", "zgreen"):
        model = bench.algorithmic_bytes(kind, n, fp, 0.8)
        assert all(m == pytest.approx(recount(kind, n, fp), rel=1e-15) for m in model)
    assert bench.algorithmic_bytes("yfwd", n, fp, 0.8) == bench.algorithmic_bytes("zgreen", n, fp, 0.8)


def test_byte_model_at_the_bench_size():
    """The figures the roofline rests on at 256^3 FP32 (GB per launch)."""
    ev, first, later = bench.algorithmic_bytes("xfwd", 256, 4, 0.8)
    assert round(ev / 1e9, 3) == 0.808 and round(first / 1e9, 2) == 1.36 and round(later / 1e9, 2) == 2.57
    assert round(bench.algorithmic_bytes("zgreen", 256, 4, 0.8)[0] / 1e9, 3) == 0.812


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stdout


def test_pass_counter_summary_derives_rocprof_metrics(tmp_path):
    """LdsBankConflict, LdsUtil, VALUBusy and the LDS-wait share from
    per-dispatch counters, with GRBM_GUI_ACTIVE summed over 8 XCDs."""
    import csv
    src = tmp_path / "pmc"
    src.mkdir()
    vals = {"SQ_LDS_BANK_CONFLICT": 100, "SQ_LDS_IDX_ACTIVE": 1100, "SQ_INSTS_LDS": 5000, "SQ_WAIT_INST_LDS": 50,
            "SQ_ACTIVE_INST_VALU": 12800, "SQ_WAVE_CYCLES": 1000, "SQ_BUSY_CYCLES": 10, "GRBM_GUI_ACTIVE": 800}
    with open(src / "run_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, name in enumerate(["void hom::k_zgreen<float, 6, 256, 2>(hom::Pipe<float>)",
                                  "void hom::k_mlp_fwd<0>(hom::FwdArgs)"]):
            for c, v in vals.items():
                w.writerow(dict(Dispatch_Id=d, Kernel_Name=name, Counter_Name=c, Counter_Value=v))
    lines = bench.pass_counter_summary(str(src), "cmd", out_path=str(tmp_path / "out.md"))
    rows = [l for l in lines if l.startswith("| hom::")]
    assert len(rows) == 1 and "k_zgreen" in rows[0]            # pass kernels only
    cells = [c.strip() for c in rows[0].strip("|").split("|")]
    # 100 / (1100 - 100); 100 * 1100 / (100 * 256); 100 * 12800 / (100 * 256); 100 * 50 / 1000
    assert cells[1:] == ["1", "5000", "0.100", "4.3", "50.0", "5.0", "100"]


def test_whole_solve_byte_model_recount():
    """solve_bytes: every kernel of the timed increments, array by array."""
    n, fp, mf, ns = 64, 4, 0.75, 79
    v = n ** 3
    comp = fp * v
    spec6 = 6 * n * n * (n // 2 + 1) * 2 * fp
    spec3 = spec6 // 2
    n_eval, n_cg, n_first, inc = 9, 40, 6, 2
    th = {"xfwd": 5, "yfwd": 5, "zgreen": 5, "yinv": 5, "xinv": 5, "init": 2, "commit": 2}
    got = bench.solve_bytes(n, fp, mf, ns, n_eval, n_cg, n_first, inc, th)
    ev, first, later = recount("xfwd", n, fp)
    assert got["xfwd"] * 1e9 == pytest.approx(n_eval * ev + n_first * first + (n_cg - n_first) * later)
    assert got["ypass"] * 1e9 == pytest.approx(2 * (n_eval + n_cg) * 2 * spec6)
    assert got["zgreen"] * 1e9 == pytest.approx((n_eval + n_cg) * 2 * spec6)
    assert got["xinv"] * 1e9 == pytest.approx((n_eval + n_cg) * (spec6 + 12 * comp))
    # evaluation: read the strain and phase, 14 FP64 of every PA66 voxel, write stress and two tangent factors;
    # after the first of an increment also the pending CG step (read p, write x)
    assert got["eval"] * 1e9 == pytest.approx(n_eval * (6 * comp + v + mf * v * 14 * 8 + 6 * comp + 2 * comp)
                                              + (n_eval - inc) * 12 * comp)
    assert got["init"] * 1e9 == pytest.approx(inc * 12 * comp)
    # history: 72 branch values in, 8 slots out, per PA66 voxel (compacted: no phase byte)
    assert got["history"] * 1e9 == pytest.approx(inc * mf * v * (72 + 8) * 8)
    # commit: x, x^n, phase in; 79 state values in and out and 8 slots in per PA66 voxel; x^n and stress out
    assert got["commit"] * 1e9 == pytest.approx(inc * (24 * comp + v + mf * v * (2 * 79 + 8) * 8))
    # conduction (3 components): x forward at the evaluation size, y, z and y^-1 passes, x inverse, init, commit
    cond = 5 * (3 * comp + spec3) + 3 * 5 * 2 * spec3 + 5 * (spec3 + 6 * comp) + 2 * 6 * comp + 2 * (3 * comp + v)
    assert got["conduction"] * 1e9 == pytest.approx(cond)
