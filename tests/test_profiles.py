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
