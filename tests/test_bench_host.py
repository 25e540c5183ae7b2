"""Host-side pieces of bench.py (no GPU): the oracle baseline and kernel naming."""
import bench
import synth


def test_cpu_baseline_runs_the_oracle_with_gpu_options_present():
    A, b, part, p = synth.workload("aniso2d_64")
    opts = dict(bench.WORKLOADS["aniso2d_64"][1], factor_prec=1)
    out = bench.cpu_baseline(A, b, None, 1, opts, 1e-8, 30, 20, 5)
    assert out["kind"] == "oracle" and out["value"] > 0 and out["cores"] >= 1
    assert "FGMRES iterations" in out["sample"]


def test_kernel_instance_names():
    # 128^3 slab layout: L_B and U_B block-local with 2 lanes of 8, L_S/U_S 1 lane of 2, one launch, all check-free
    sched = [1, 2, 8, 256, 1, 2, 8, 256, 1, 1, 2, 256, 1, 1, 2, 256, 1, 15, 0, 0]
    assert bench.kernel_instance("trsv_LB_W", sched) == "void silu::k_trsv_lds<2, 8, false, 0, true>"
    assert bench.kernel_instance("trsv_UB_Z", sched, 1) == "void silu::k_trsv_lds<2, 8, true, 1, true>"
    assert bench.kernel_instance("trsv_LS", sched) == "void silu::k_trsv_lds_pair<1, 2, 0, true>"
    sched[17] = 1  # only L_B check-free
    assert bench.kernel_instance("trsv_LS", sched, 2) == "void silu::k_trsv_lds_pair<1, 2, 2, false>"
    assert bench.kernel_instance("mgs", sched) == "void silu::k_mgs_step<"
