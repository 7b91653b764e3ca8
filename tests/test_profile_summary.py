"""Host logic of the rocprofv3 summary tool (no GPU): kernel-name parsing and
the copy-calibrated traffic figures."""

import csv

import pytest

from paper_1907_05560_amd import profile_summary as PS

NS = "nuosc::(anonymous namespace)::"


def _final(ts, t, arg="RunConst", kernel="k_final_one", nj=2):
    return f"void {NS}{kernel}<{ts}, {t}, 3, {NS}TabDP54, {nj}>(nuosc::{arg})"


@pytest.mark.parametrize("kernel,arg", [("k_final_one", "RunConst"), ("k_final", "LaunchSet")])
@pytest.mark.parametrize("ts,t", [("double", "double"), ("float", "float"), ("float", "double")])
def test_kernel_key_drops_the_single_run_suffix(kernel, arg, ts, t):
    n = _final(ts, t, arg, kernel)
    assert PS.short_name(n) == f"{kernel}<{ts},{t},3,DP54,2>"
    assert PS.kernel_key(n) == f"k_final<{ts},{t},3,DP54,2>"


def test_kernel_keys_of_the_other_launches():
    traj = f"void {NS}k_traj_one<3, {NS}TabDP54, 2, 4, float>(nuosc::RunConst)"
    power = f"void {NS}k_power_one<float, 3, {NS}TabDP54, 2, false>(nuosc::RunConst)"
    assert PS.kernel_key(traj) == "k_traj<3,DP54,2,4,float>"
    assert PS.kernel_key(power) == "k_power<float,3,DP54,2,false>"
    assert PS.kernel_key(PS.COPY_KERNEL) == PS.COPY_KERNEL


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_is_scaled_by_the_calibration_copy(tmp_path):
    k6 = _final("float", "float")
    mib = 64
    # the copy reads 2 x its size by FETCH_SIZE and writes 1 x by WRITE_SIZE
    f_rows = [(PS.COPY_KERNEL, 2 * mib * 1024), (k6, 1000.0), (k6, 1000.0), (k6, 10.0)]  # last: early exit
    w_rows = [(PS.COPY_KERNEL, mib * 1024), (k6, 500.0), (k6, 500.0), (k6, 5.0)]
    fp, wp = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fp, "FETCH_SIZE", f_rows)
    _write(wp, "WRITE_SIZE", w_rows)
    text, doc = PS.traffic_summary(str(fp), str(wp), mib, "cmd f", "cmd w")
    assert doc["fetch_scale"] == pytest.approx(0.5)
    assert doc["write_scale"] == pytest.approx(1.0)
    assert doc["bytes_per_launch"]["k_final<float,float,3,DP54,2>"] == round(1000 * 1024 * 0.5 + 500 * 1024)
    assert "k_final_one<float,float,3,DP54,2>" in text


def test_valu_summary_reads_the_exponential_stepper_launches(tmp_path):
    def nm(L):
        return f"void {NS}k_exp_beam<3, {L}>(nuosc::RunConst)"

    rows = [(nm(1), 1000.0), (nm(1), 1000.0), (nm(3), 3000.0), (nm(0), 50.0), (nm(2), 2000.0), (nm(2), 10.0)]
    path = tmp_path / "v.csv"
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, value in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": "SQ_INSTS_VALU", "Counter_Value": value})
            w.writerow({"Kernel_Name": name, "Counter_Name": "SQ_WAVES", "Counter_Value": 10.0})
    text, doc = PS.valu_summary(str(path), "cmd")
    assert doc["valu_wave_instr_per_launch"] == {"launch1": 1000, "launch2": 2000, "launch3": 3000}
    assert doc["source_sha256_16"] == PS.exp_source_hash()
    assert "k_exp_beam<3,2>" in text and PS.exp_launch(nm(0)) is None
