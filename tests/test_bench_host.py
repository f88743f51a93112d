"""Host logic of bench.py: the exact nonzero count of A that the roofline's
algorithmic figure uses (against the oracle's dense A: entries whose chord is
longer than 1e-12; a ray that only grazes a pixel corner has length zero in
exact arithmetic), and the reading of the committed rocprofv3 summaries,
which must be dropped once the kernel sources differ from the ones they
were taken with."""
import hashlib
import re

import numpy as np
import pytest

import bench


@pytest.mark.parametrize("geom", [(16, 24, 25), (17, 30, 26), (33, 45, 49), (20, 7, 12),
                                  (9, 1, 13), (64, 90, 95)])
def test_count_nnz_is_the_dense_count(oracle_lib, geom):
    A = oracle_lib.Geometry(*geom).dense()
    assert bench.count_nnz(*geom) == int(np.count_nonzero(A > 1e-12))


def _sources_sha():
    h = hashlib.sha256()
    for f in bench.KERNEL_SOURCES:
        h.update(open(f, "rb").read())
    return h.hexdigest()


def _copy_with_sha(src, dst, sha):
    text = open(src).read()
    open(dst, "w").write(re.sub(r"sha256: [0-9a-f]{64}", "sha256: " + sha, text))


def test_summaries_follow_the_sources(tmp_path, monkeypatch):
    cur = _sources_sha()
    op = tmp_path / "op.md"
    bt = tmp_path / "bt.md"
    _copy_with_sha(bench.TRAFFIC_FILE, op, cur)
    _copy_with_sha(bench.BATCHED_TRAFFIC_FILE, bt, cur)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(op))
    monkeypatch.setattr(bench, "BATCHED_TRAFFIC_FILE", str(bt))
    t = bench.measured_traffic("kb_project")
    assert isinstance(t, int) and t > 0
    r = bench.batched_roofline()
    assert r is not None and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["kernel"] in bench.STREAMING_HBM
    for k, v in r["per_kernel"].items():
        assert v["frac"] == pytest.approx(v["algorithmic_bytes"] / (v["avg_us"] * 1e-6)
                                          / bench.PEAK_HBM)
    # another source text: both readings are dropped
    _copy_with_sha(bench.TRAFFIC_FILE, op, "0" * 64)
    _copy_with_sha(bench.BATCHED_TRAFFIC_FILE, bt, "0" * 64)
    assert bench.measured_traffic("kb_project") is None
    assert bench.batched_roofline() is None

