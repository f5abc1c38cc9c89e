"""Host-side measurement logic (CPU): the rocprofv3 summaries and traffic lookup of
paper_2011_01207_amd.profiling, and the benchmark's roofline assembly from stage timings."""
import csv
import importlib.util
import os

import pytest

from paper_2011_01207_amd import profiling

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TILES = "k_block_tiles<float, true, DipoleKind<float>, false, 0>"
TILES_RAW = "void amoeba::k_block_tiles<float, true, amoeba::DipoleKind<float>, false, 0>(int, ...)"


def write_csv(path, header, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def counter_rows(copy_kib, tiles_kib, n_tiles=3):
    rows = [[profiling.COPY_KERNEL, 67108864, v] for v in (copy_kib, copy_kib, copy_kib)]
    rows += [[TILES_RAW, 384000, tiles_kib] for _ in range(n_tiles)]
    return rows


def test_traffic_is_copy_calibrated_and_keyed_by_the_sources(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Value"]
    # the copy of 256 MiB reads 2^18 KiB; FETCH reports half of it, WRITE all of it
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    write_csv(fetch, hdr, counter_rows(131072.0, 1000.0))
    write_csv(write, hdr, counter_rows(262144.0, 500.0))
    md = profiling.traffic_md(str(fetch), str(write), "t", "cf", "cw")
    expect = 1000.0 * 1024 * 2.0 + 500.0 * 1024 * 1.0
    path = tmp_path / "traffic.md"
    path.write_text(md)
    assert profiling.traffic_lookup(str(path), TILES) == pytest.approx(expect)
    # a different source hash in the row: the summary no longer describes the kernel
    stale = md.replace(profiling.source_hash(profiling.sources_of(TILES)), "0123456789abcdef")
    path.write_text(stale)
    assert profiling.traffic_lookup(str(path), TILES) is None
    assert profiling.traffic_lookup(str(tmp_path / "missing.md"), TILES) is None


def test_traffic_needs_the_copy_calibration(tmp_path):
    hdr = ["Kernel_Name", "Grid_Size", "Counter_Value"]
    f = tmp_path / "f.csv"
    write_csv(f, hdr, [[TILES_RAW, 384000, 10.0]])
    with pytest.raises(SystemExit):
        profiling.traffic_md(str(f), str(f), "t", "a", "b")


def test_stream_table_separates_working_dispatches(tmp_path):
    hdr = ["Kernel_Name", "Stream_Id", "Start_Timestamp", "End_Timestamp"]
    rows = [[TILES_RAW, 1, 0, 60000], [TILES_RAW, 1, 0, 2000], [TILES_RAW, 0, 0, 50000],
            ["void amoeba::k_update(int)", 0, 0, 7000]]
    p = tmp_path / "trace.csv"
    write_csv(p, hdr, rows)
    md = profiling.streams_md(str(p))
    lines = [l for l in md.splitlines() if l.startswith("| `k_block_tiles")]
    assert len(lines) == 2
    cols = {l.split("|")[2].strip(): [c.strip() for c in l.split("|")[3:7]] for l in lines}
    assert cols["0"] == ["1", "50.00", "1", "50.00"]
    assert cols["1"] == ["2", "31.00", "1", "60.00"]


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def timing(real_ms, launches, matvecs, other_ms=1.0):
    ms = {k: other_ms for k in ("list", "perm", "real", "spread", "fft", "gather", "pcg", "guess")}
    ms["real"] = real_ms
    n = {k: launches for k in ms}
    return {"ms": ms, "launches": n, "matvecs": matvecs}


def test_roofline_uses_the_live_tile_time():
    bench = load_bench()

    class S:
        n = 1000
        grid = (8, 8, 8)
        name = "test_box"

    # 100 PCG products and 10 basis products of a learned start are productive; the other
    # launches returned at entry after convergence
    res = {"timing": timing(10.0, 120, 100), "timing_live": timing(12.5, 120, 100, other_ms=0.0),
           "n_pairs": 1_000_000, "n_tiles": 100, "pme_planes": 1, "pair_min_image": 0, "pair_store": 0,
           "extra_real_products": 10}
    top, stages = bench.roofline(S, res)
    flops = bench.FLOPS_PER_PAIR * 1_000_000 * 110
    assert top["stage"] == "real" and top["kernel"] == TILES
    assert top["achieved"] == pytest.approx(flops / 12.5e-3 / 1e12)
    assert top["achieved_alone"] == pytest.approx(flops / 10.0e-3 / 1e12)
    assert top["avg_launch_us"] == pytest.approx(12.5e3 / 120)
    assert top["productive_launches"] == 110
    assert top["frac"] == pytest.approx(top["achieved"] / bench.PEAK_FP32_VALU)
    assert top["frac_nonpacked"] == pytest.approx(top["achieved"] / bench.PEAK_FP32_NONPACKED)
    # without a live timing the stage pass is reported
    res.pop("timing_live")
    top2, _ = bench.roofline(S, res)
    assert top2["achieved"] == pytest.approx(flops / 10.0e-3 / 1e12)
    assert "achieved_alone" not in top2


def test_step_statistics():
    bench = load_bench()
    st = bench.pstats([5.0, 1.0, 2.0, 4.0, 3.0])
    assert st["median_ms"] == 3.0 and st["mean_ms"] == 3.0
    assert st["p10_ms"] == pytest.approx(1.4) and st["p90_ms"] == pytest.approx(4.6)
