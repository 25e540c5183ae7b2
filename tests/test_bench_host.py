"""Host-side pieces of bench.py (no GPU): the oracle baseline and kernel naming."""
import bench
import synth


def test_cpu_baseline_runs_the_oracle_in_worker_processes():
    # the oracle runs in child processes (one alone, then two at once), each on the bounded sample
    out = bench.cpu_baseline("aniso2d_64", "f32", 20, 5, 2)
    assert out["kind"] == "oracle" and out["cores"] == 2
    assert out["value"] > out["one_core_value"] > 0
    assert "FGMRES iterations" in out["sample"] and out["cpu_model"]


def test_kernel_instance_names():
    # 128^3 slab layout: L_B and U_B block-local with 2 lanes of 8, L_S/U_S 1 lane of 2, one launch, all check-free
    sched = [1, 2, 8, 256, 1, 2, 8, 256, 1, 1, 2, 256, 1, 1, 2, 256, 1, 15, 0, 0]
    assert bench.kernel_instance("trsv_LB_W", sched) == "void silu::k_trsv_lds<2, 8, false, 0, true>"
    assert bench.kernel_instance("trsv_UB_Z", sched, 1) == "void silu::k_trsv_lds<2, 8, true, 1, true>"
    assert bench.kernel_instance("trsv_LS", sched) == "void silu::k_trsv_lds_pair<1, 2, 0, true>"
    sched[17] = 1  # only L_B check-free
    assert bench.kernel_instance("trsv_LS", sched, 2) == "void silu::k_trsv_lds_pair<1, 2, 2, false>"
    assert bench.kernel_instance("mgs", sched) == "void silu::k_arnoldi<"
    assert bench.kernel_instance("spmv_A", sched) == "void silu::k_spmv<0>"
    assert bench.kernel_instance("spmv_Coff", sched) == "void silu::k_spmv<1>"
    # L_B and U_B split over two workgroups per subdomain (schedule entries 20 and 21)
    split = sched[:17] + [15, 0, 0, 2, 2]
    assert bench.kernel_instance("trsv_LB_W", split) == "void silu::k_trsv_lds_x<2, 8, false, 0>"
    assert bench.kernel_instance("trsv_UB_Z", split, 1) == "void silu::k_trsv_lds_x<2, 8, true, 1>"
    assert bench.kernel_instance("trsv_UB_Z", sched[:17] + [15, 0, 0, 2, 1]) == \
        "void silu::k_trsv_lds<2, 8, true, 0, true>"
