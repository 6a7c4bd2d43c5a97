"""Host-side logic of the library checked without a GPU: the eigensolver's
index helpers (tournament pairings, NaN-safe ordering) compiled with g++ from
the same header the kernels include."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_jacobi_index_logic(tmp_path):
    exe = tmp_path / "jacobi_order"
    src = os.path.join(ROOT, "tests", "cpp", "test_jacobi_order.cpp")
    inc = os.path.join(ROOT, "paper_2211_07894_amd", "csrc")
    subprocess.run(["g++", "-O2", "-std=c++17", f"-I{inc}", src, "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_traffic_summary_scales_by_calibration_copy(tmp_path):
    """HBM bytes per dispatch = counted KiB x 1024 x (1 GiB / counted bytes of the
    calibration copy); median over the dispatches of each kernel."""
    from paper_2211_07894_amd import profile_summary as ps

    def write(path, counter, rows):
        with open(path, "w") as f:
            f.write("Dispatch_Id,Kernel_Name,Counter_Name,Counter_Value\n")
            for d, name, v in rows:
                f.write(f'{d},"{name}",{counter},{v}\n')

    gib_kib = (1 << 30) / 1024
    copy = "void at::native::vectorized_elementwise_kernel<4, MulFunctor>(int)"
    proj = "void lrdm::(anonymous namespace)::tn_sym_pipe_kernel<(lrdm::(anonymous namespace)::Core)2, true>(float const*)"
    back = "void lrdm::(anonymous namespace)::backproj_pipe_kernel<(lrdm::(anonymous namespace)::Core)2>(float const*)"
    write(tmp_path / "f.csv", "FETCH_SIZE",
          [(1, copy, 1.25 * gib_kib), (2, copy, 1.25 * gib_kib), (3, copy, 1.25 * gib_kib),
           (4, proj, 1000.0), (5, proj, 1000.0), (6, proj, 4000.0), (7, back, 500.0)])
    write(tmp_path / "w.csv", "WRITE_SIZE",
          [(1, copy, gib_kib), (2, copy, gib_kib), (3, copy, gib_kib),
           (4, proj, 10.0), (5, proj, 10.0), (6, proj, 10.0), (7, back, 20.0)])
    recs = {r["kernel"]: r for r in ps.traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"),
                                               "bf16x3", "wl", "cmd")}
    assert set(recs) == {"proj", "backproj"}
    assert recs["proj"]["fetch_bytes_per_launch"] == round(1000.0 * 1024 / 1.25)
    assert recs["proj"]["write_bytes_per_launch"] == round(10.0 * 1024)
    assert recs["backproj"]["bytes_per_launch"] == round(500.0 * 1024 / 1.25) + round(20.0 * 1024)
    assert recs["proj"]["source"] == "gemm_lp.hip" and len(recs["proj"]["source_sha"]) == 16


def test_lrdma_driver_gates_are_the_papers():
    """The GPU driver's LRDMA decision against the parameters Sec. III A prints
    (golden fixture): accumulation only while ||R|| < 1.0, CL above beta 0.1."""
    from paper_2211_07894_amd.scf import lrdma_event
    from tests.pins import sec3a_parameters
    p = sec3a_parameters()
    gate, btol, s_tol = (p["lrdma_accumulate_only_below_norm_R"], p["lrdma_beta_tol"],
                         p["s_tol_range"][1])

    def ev(kept=3, pending=False, beta=0.0, s_rel=0.9, nR=0.5):
        return lrdma_event(kept, pending, beta, s_rel, nR, s_tol, btol, gate)
    assert ev(nR=1.5) == "CR" and ev(nR=gate) == "CR" and ev(nR=0.999) == "accumulate"
    assert ev(beta=0.11) == "CL" and ev(s_rel=0.1, nR=1.5) == "reuse"
    assert ev(pending=True) == "CT" and ev(kept=0) == "fresh"


def test_lowrank_params_defaults_are_the_papers():
    """LowRankParams defaults: alpha 0.1 until ||R|| goes below 2.0, then 0.5."""
    from paper_2211_07894_amd import LowRankParams
    from tests.pins import sec3a_parameters
    p, d = sec3a_parameters(), LowRankParams()
    assert (d.alpha_far, d.alpha_near, d.alpha_switch) == (
        p["alpha_far"], p["alpha_near"], p["alpha_switch_below_norm_R"])
    assert p["s_tol_range"][0] <= d.s_tol <= p["s_tol_range"][1]

