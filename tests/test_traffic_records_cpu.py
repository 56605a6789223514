"""The committed HBM-traffic records of the dominant kernels (profiles/traffic_*.json, written
from rocprofv3 FETCH_SIZE / WRITE_SIZE runs by `bench.py --traffic-from`) were taken on the
kernel sources as they are: each carries the hash of those sources, and bench.py reports the
traffic only while the hash matches.  A kernel edit without new counters fails here (CPU only)."""
import glob
import importlib.util
import json
import os

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_traffic_records_match_the_kernel_sources():
    b = _bench()
    records = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")))
    assert records, "no traffic records"
    now = b.kernel_source_hash()
    for path in records:
        rec = json.load(open(path))
        assert rec["kernel_source_hash"] == now, (
            f"{os.path.basename(path)} was taken on kernel sources {rec['kernel_source_hash']}, "
            f"now {now}: re-take FETCH_SIZE / WRITE_SIZE")
        assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"]


def test_headline_record_exists():
    b = _bench()
    for L in (0, 2):
        assert os.path.exists(b.traffic_path(L, "abc", 16384)), L
