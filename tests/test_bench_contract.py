"""Host-side checks of the benchmark script's contract (no GPU needed).

* More than one GPU is refused with a message and a non-zero exit, before any
  GPU work (there is no multi-GPU path).
* The algorithmic byte model: each finest-level kernel class counts every
  array once (FP64 residual 33 B/cell: x, b, k read, r written, 1/8 cell of
  restricted residual; the two-sweep pass 33 B/cell: 1/8 cell of coarse
  correction, r, k and x read, x written), and a whole cycle adds the coarse
  levels, each 1/8 of the one above, so the per-cell total stays between the
  finest-level bytes and 8/7 of them.
* The roofline object carries the fields the report format names.
"""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in p.stderr


def test_finest_level_bytes_per_cell():
    f = bench.BYTES_PER_CELL
    # FP64 direct form: the residual kernel reads x, b, k and writes R r only
    assert f["fp64"]["resid"] == 8 + 8 + 8 + 1
    assert f["fp64"]["sweeps"] == 1 + 8 + 8 + 8 + 8
    assert f["fp64c"]["resid"] == f["fp64"]["resid"] - 8  # no coefficient
    assert f["mixed"]["sweeps"] - f["fp16"]["sweeps"] == 2  # FP32 vs FP16 coefficient
    for mode in f:
        assert set(f[mode]) == set(bench.KCLASS)
    # the 8^3 block form writes and reads the full residual r
    g = bench.BYTES_PER_CELL_BLOCK
    for mode in g:
        assert g[mode]["resid"] == f[mode]["resid"] + 8
        assert g[mode]["sweeps"] == f[mode]["sweeps"]


def test_fine_bytes_follows_the_finest_sweep_form():
    march = {"tiles": [[[64, 2, 16], [32, 2, 16], [64, 2, 16]]]}
    block = {"tiles": [[[64, 2, 16], [8, 8, 8], [64, 2, 16]]]}
    assert bench.fine_bytes("fp64", march) is bench.BYTES_PER_CELL["fp64"]
    assert bench.fine_bytes("fp64", {"tiles": None}) is bench.BYTES_PER_CELL["fp64"]
    assert bench.fine_bytes("fp64", block) is bench.BYTES_PER_CELL_BLOCK["fp64"]
    assert bench.fine_bytes("mixed", block) is bench.BYTES_PER_CELL["mixed"]


def test_cycle_bytes_geometric_in_levels():
    levels = [(256 >> l,) * 3 for l in range(7)]
    n0 = 256 ** 3
    for mode in ("fp64", "mixed", "fp16", "fp64c"):
        per_cell = bench.cycle_model_bytes({"levels": levels}, mode) / n0
        fine = bench.BYTES_PER_CELL[mode]["resid"] + bench.BYTES_PER_CELL[mode]["sweeps"]
        assert fine < per_cell < fine * 8.0 / 7.0
    # one level: the finest kernels only
    assert bench.cycle_model_bytes({"levels": levels[:1]}, "fp64") == n0 * 58


def test_roofline_fields():
    res = {"n": 256 ** 3, "kern": {"resid": (10, 1.2), "sweeps": (10, 2.0), "sweep": (0, 0.0)}}
    best, roof, per_kernel = bench.roofline(res, "fp64", {"sweeps": 6.0e8})
    assert best == "sweeps"
    assert set(roof) == {"bound", "achieved", "peak", "unit", "frac", "traffic"}
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    want = 33 * 256 ** 3 / (2.0 / 10 / 1e3) / 1e9
    assert abs(roof["achieved"] - round(want, 1)) < 0.06
    assert abs(roof["frac"] - want / 8000.0) < 1e-4
    assert roof["traffic"] == 6.0e8
    assert "sweep" not in per_kernel  # classes that did not run are left out


def test_measured_traffic_tied_to_kernel_sources():
    # the counter figures hold only for the kernel sources and the launch form
    # (bytes per cell) they were taken on
    cur = {cls: bench.kernel_source_hash(cls) for cls in bench.KERNEL_SOURCES}
    bpc = bench.BYTES_PER_CELL["fp64"]
    table = {cls: (1.0e9, cur[cls], bpc[cls]) for cls in cur}
    assert bench.measured_traffic(table, bpc) == {cls: 1.0e9 for cls in cur}
    stale = dict(table, sweeps=(1.0e9, "0" * 16, bpc["sweeps"]))
    got = bench.measured_traffic(stale, bpc)
    assert "sweeps" not in got and got["resid"] == 1.0e9
    other_form = dict(table, resid=(1.0e9, cur["resid"], bpc["resid"] + 8))
    got = bench.measured_traffic(other_form, bpc)
    assert "resid" not in got and got["sweeps"] == 1.0e9
    # the committed figures name classes the bench knows
    assert set(bench.MEASURED_TRAFFIC_FP64_256) <= set(bench.KERNEL_SOURCES)
