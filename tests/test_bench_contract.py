"""Host checks of bench.py's measurement plumbing: the one-GPU guard, the
roofline arithmetic, the rocprofv3 counter summary, and the committed HBM
traffic records (current for the kernel source, scaled consistently, close
to the algorithmic bytes)."""

import glob
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and not r.stdout.strip()


def test_roofline_takes_the_largest_site_per_launch():
    prof = [dict(name="w", level=1, launches=2, ms=0.10, bytes=2 * 300e6, workgroups=7, block=256),
            dict(name="down", level=1, launches=2, ms=0.16, bytes=2 * 400e6, workgroups=7, block=256),
            dict(name="interp", level=0, launches=1, ms=0.05, bytes=100e6, workgroups=9, block=256)]
    dom, roof = bench.roofline(prof)
    assert dom["name"] == "down"
    assert roof["ms_per_launch"] == pytest.approx(0.08)
    assert roof["bytes_per_launch"] == pytest.approx(400e6)
    assert roof["achieved"] == pytest.approx(400e6 / 0.08e-3 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], abs=1e-4)
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0


def test_pmc_summary_averages_per_kernel_and_launch_size(tmp_path):
    csv = tmp_path / "run_counter_collection.csv"
    csv.write_text("Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n"
                   "void amgdd::dev::k_relax<double>(x),1856256,256,FETCH_SIZE,100\n"
                   "void amgdd::dev::k_relax<double>(x),1856256,256,FETCH_SIZE,300\n"
                   "void amgdd::dev::k_w<double>(x),2560,256,FETCH_SIZE,7\n")
    out = bench.summarize_pmc(str(csv))
    line = [l for l in out.splitlines() if l.startswith("k_relax<double>")][0]
    assert line.split()[1] == "7251" and line.split()[-2] == "2" and float(line.split()[-1]) == 200.0


def _records():
    return sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))


def test_traffic_records_are_consistent_and_used_only_while_current():
    """Every record's arithmetic is consistent; bench.py reports a record's
    traffic only while the kernel source it was measured on is the current
    one (a stale record gives traffic = null)."""
    recs = _records()
    assert recs, "no traffic record in profiles/"
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1906_10575_amd", "csrc", "kernels.hpp"), "rb").read()).hexdigest()
    for path in recs:
        r = json.load(open(path))
        dom = dict(name=r["site"], level=r["level"], workgroups=r["workgroups"])
        if r["kernels_sha256"] != sha:
            assert bench.measured_traffic(dom) is None
            continue
        cal = r["calibration"]
        assert cal["fetch_factor"] == pytest.approx(cal["fetch_size_kib"] / cal["expected_kib"], abs=1e-4)
        assert cal["write_factor"] == pytest.approx(cal["write_size_kib"] / cal["expected_kib"], abs=1e-4)
        t = (r["fetch_size_kib"] / cal["fetch_factor"] + r["write_size_kib"] / cal["write_factor"]) * 1024
        assert r["traffic_bytes"] == pytest.approx(t, rel=1e-3)
        # operator passes stay near their algorithmic bytes; the reordered
        # interpolation and restriction rows carry slice padding (up to ~2.2x)
        assert 0.95 <= r["traffic_bytes"] / r["algorithmic_bytes"] <= 2.5
        if r["site"] in ("relax_post", "w", "down") and r["level"] <= 4:
            assert r["traffic_bytes"] / r["algorithmic_bytes"] <= 1.2
        # bench.py finds the record for its launch site
        assert bench.measured_traffic(dom) == r["traffic_bytes"]


def test_cpu_baseline_times_the_oracle_on_the_sample():
    rec = bench.cpu_baseline(seconds=0.5)
    assert rec["kind"] == "oracle" and rec["unit"] == "DOF*cycles/s"
    assert rec["value"] > 0 and rec["one_core"]["value"] > 0 and rec["one_core"]["cores"] == 1
    share, host = bench.host_cores()
    assert rec["cores"] == min(share, 27) and host["affinity"] >= 1
    assert "72^3" in rec["sample"]


def test_traffic_records_from_counter_output(tmp_path):
    """FETCH_SIZE / WRITE_SIZE per dispatch, scaled by the calibration kernel's
    counters (256 MiB read and written), matched to the --sites log by kernel
    and workgroup count."""
    head = "Kernel_Name,Grid_Size,Workgroup_Size,Counter_Name,Counter_Value\n"
    cal = '"void at::native::vectorized_elementwise_kernel<4, at::native::CUDAFunctorOnSelf_add<double> >(x)",8388608,256,{c},{v}\n'
    fill = '"void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<double> >(x)",8388608,256,{c},12.5\n'
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    fetch.write_text(head + cal.format(c="FETCH_SIZE", v=131072.0) + fill.format(c="FETCH_SIZE") +
                     '"void amgdd::dev::k_w<double, 256>(x)",11389696,256,FETCH_SIZE,1000000\n'
                     '"void amgdd::dev::k_w<double, 256>(x)",11389696,256,FETCH_SIZE,1100000\n'
                     '"void amgdd::dev::k_relax<double, 256>(x)",11389696,256,FETCH_SIZE,999\n')
    write.write_text(head + cal.format(c="WRITE_SIZE", v=262144.0) +
                     '"void amgdd::dev::k_w<double, 256>(x)",11389696,256,WRITE_SIZE,90000\n')
    log = tmp_path / "sites.err"
    log.write_text("[bench] site           lvl  n  ms/iter   MB/iter    GB/s     wg\n"
                   "[bench] w                1  2   0.8686    4126.3    4750  44491\n"
                   "[bench] relax_post       1  2   0.1000    1000.0    4750  44491\n")
    recs = bench.traffic_records(str(fetch), str(write), str(log), "cfg3", top=1)
    assert len(recs) == 1 and recs[0]["site"] == "w" and recs[0]["workgroups"] == 44491
    # fetch factor 0.5: 1.05e6 KiB counted = 2.1e6 KiB read; write factor 1
    assert recs[0]["traffic_bytes"] == round((1.05e6 / 0.5 + 90000.0) * 1024)
    assert recs[0]["algorithmic_bytes"] == 4126.3e6 / 2
    # every named site of chosen levels, with the third counter pass
    extra = tmp_path / "x.csv"
    rows = {"GRBM_GUI_ACTIVE": 800000, "TA_TA_BUSY": 256 * 50000, "TA_ADDR_STALLED_BY_TC_CYCLES": 256 * 10000,
            "TCP_TCC_READ_REQ": 2000000, "TCP_TCC_READ_REQ_LATENCY": 1.6e9, "SQ_WAVES": 100,
            "SQ_WAVE_CYCLES": 1000, "SQ_WAIT_INST_ANY": 400}
    extra.write_text(head + "".join(f'"void amgdd::dev::k_w<double, 256>(x)",11389696,256,{k},{v}\n'
                                    for k, v in rows.items()))
    recs = bench.traffic_records(str(fetch), str(write), str(log), "cfg3", levels={1}, names={"w"},
                                 extra_csv=str(extra))
    assert [r["site"] for r in recs] == ["w"]
    ex = recs[0]["l1_l2_path"]
    assert ex["l2_read_latency_cycles"] == 800.0
    assert ex["ta_busy_frac"] == pytest.approx(50000 / 100000, abs=1e-3)  # 800000 / 8 XCDs = 100000 cycles
    assert ex["ta_stalled_by_l1_frac"] == pytest.approx(0.1, abs=1e-3)
    assert ex["wave_wait_frac"] == 0.4
    assert recs[0]["traffic_over_algorithmic"] == pytest.approx(recs[0]["traffic_bytes"] / recs[0]["algorithmic_bytes"],
                                                                abs=1e-3)
