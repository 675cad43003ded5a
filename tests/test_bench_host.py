"""Host-side helpers of bench.py (CPU): the label-fixture reader, the
counter-summary lookup behind the roofline's `traffic`, and the refusal of
more than one GPU.  No GPU work runs here."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(HERE, "golden"))

import bench  # noqa: E402
import make_prescreen_labels as mk  # noqa: E402


def test_label_reader_expands_hex_rows():
    recipe, rows = bench._load_labels("prescreen_labels_2p20.txt")
    assert recipe == mk.RECIPE_2P20
    assert len(rows) == 10240 and all(len(b) == 256 for _, b in rows)
    # the hex form of a row is its bit string, block 0 in the leading bit
    with open(os.path.join(HERE, "golden", "prescreen_labels_2p20.txt")) as f:
        raw = {int(a): b for a, b in (l.split() for l in f if l.strip() and not l.startswith("#"))}
    for i, bits in rows[:64]:
        assert int(raw[i], 16) == int(bits, 2)
    # the 2^16 fixture is read unchanged (one 0/1 per block)
    recipe16, rows16 = bench._load_labels("prescreen_labels.txt")
    assert recipe16 == mk.RECIPE and all(len(b) == 16 for _, b in rows16)


def test_traffic_is_reported_only_for_matching_sources():
    for f in ("k_ols_conv.hip", "k_harmsum.hip"):
        assert isinstance(bench.read_traffic(f, "bytes_per_launch"), int), f
    assert bench.read_traffic("k_direct_conv.hip", "bytes_per_launch") is None  # no counters recorded
    # a summary whose digest no longer matches the source is stale
    real = bench.kernel_source_digest
    try:
        bench.kernel_source_digest = lambda name: "0000000000000000"
        assert bench.read_traffic("k_ols_conv.hip", "bytes_per_launch") is None
    finally:
        bench.kernel_source_digest = real


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
