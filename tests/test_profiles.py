"""The committed rocprofv3 summaries parse, and the bench's traffic lookup reads them."""
import glob
import os

from paper_2311_03096_amd import prof_summary as ps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_short_names():
    assert ps.short_name("void wsr::k_prox_fwd_small<4096, 512>(wsr::SegArgs, float const*)") == "prox_fwd_small_4096"
    assert ps.short_name("wsr::k_radix_scatter(float const*, unsigned int const*)") == "radix_scatter"
    assert ps.short_name("void wsr::k_big_merge<16, 8>(int, int)") == "big_merge"


def test_traffic_summaries_parse():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.md")))
    assert files, "no traffic summaries committed"
    for f in files:
        workload = os.path.basename(f)[len("traffic_"):-len(".md")]
        recs = [l for l in open(f) if l.startswith("traffic-record:")]
        assert recs, f
        for line in recs:
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            assert kv["workload"] == workload
            assert float(kv["read_bytes"]) >= 0 and float(kv["write_bytes"]) >= 0
            assert len(kv["src"]) == 16
        assert "rocprofv3 --pmc FETCH_SIZE" in open(f).read()


def test_read_traffic_rejects_other_sources(tmp_path):
    p = tmp_path / "traffic_x.md"
    p.write_text("traffic-record: workload=x kernel=k src=0000000000000000 read_bytes=10 write_bytes=5\n")
    assert ps.read_traffic(str(p), "x", "k") is None  # measured on other kernel sources
    p.write_text("traffic-record: workload=x kernel=k src=%s read_bytes=10 write_bytes=5\n" % ps.source_hash())
    assert ps.read_traffic(str(p), "x", "k") == 15.0
    assert ps.read_traffic(str(p), "x", "other") is None


def test_counter_summary_parses():
    f = os.path.join(ROOT, "profiles", "counters_mlp_rows.md")
    recs = [l for l in open(f) if l.startswith("counter-record:")]
    assert recs
    for line in recs:
        kv = dict(t.split("=", 1) for t in line.split()[1:])
        assert kv["workload"] == "mlp_rows" and len(kv["src"]) == 16
        assert float(kv["valu"]) > 0 and float(kv["waves"]) > 0
    assert "rocprofv3 --pmc SQ_INSTS_VALU" in open(f).read()


def test_phase_summary_reduces_timestamps():
    """The bench's reduction of phase timestamps: durations, shares, span and resident workgroups
    on a hand-checked example (workgroups that never reached the last mark are left out)."""
    import numpy as np
    import bench
    t = np.array([[0, 10, 30, 40, 70, 80, 0, 0],
                  [40, 50, 60, 70, 80, 100, 0, 0],
                  [90, 100, 110, 120, 130, 140, 0, 0],
                  [5, 6, 0, 0, 0, 0, 0, 0]], dtype=np.float64)
    names = ("a", "b", "c", "d", "e")
    r = bench.phase_summary(t, names, 0.01, 1)
    assert r["span_us"] == 1.4
    assert r["workgroup_us_mean"] == round((0.8 + 0.6 + 0.5) / 3, 2)
    assert r["in_flight_max_per_cu"] == 2.0  # [0, 80] and [40, 100] overlap, [90, 140] with the second
    assert r["in_flight_per_cu"] == round((80 + 60 + 50) / 140, 2)
    assert r["a"]["us_mean"] == 0.1 and r["a"]["share"] == round(30 / 190, 3)
    assert r["d"]["us_mean"] == round((0.3 + 0.1 + 0.1) / 3, 2)
    assert abs(sum(r[n]["share"] for n in names) - 1.0) < 5e-3
    # a workgroup that ends exactly where another starts does not count as overlapping it
    r2 = bench.phase_summary(np.array([[0, 1, 2, 3, 4, 5], [5, 6, 7, 8, 9, 10]], dtype=np.float64), names, 1.0, 1)
    assert r2["in_flight_max_per_cu"] == 1.0
