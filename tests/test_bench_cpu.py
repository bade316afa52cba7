"""Host logic of the benchmark's roofline (no GPU): the algorithmic bytes of
each level-pass launch and the measured-traffic lookup for the dominant
level-pass kernel."""
import json

import pytest

import bench


def test_level_pass_bytes_byte_alphabet_lastbits():
    n, L = 1 << 28, 8
    per = bench.level_pass_bytes(n, L, 1, 1, L, lastbits=True)
    dirs = n / 8 + n / 64 + n / 256
    # levels 0..L-3: read the level's sequence, write the next one, bits and directories
    assert per[:L - 2] == [2 * n + dirs] * (L - 2)
    # level L-2: no sequence written, the last level's bits instead
    assert per[L - 2] == n + dirs + n / 8
    # the last level: its bits read back for the directories
    assert per[L - 1] == n / 8 + dirs
    # the dominant kernel's figure: 2.1445... bytes per symbol
    assert per[0] / n == pytest.approx(2 + 1 / 8 + 1 / 64 + 1 / 256)


def test_level_pass_bytes_pairs_and_wide():
    n = 1000
    dirs = n / 8 + n / 64 + n / 256
    # two levels per pass, L = 5: pairs (0,1), (2,3), then level 4 alone
    assert bench.level_pass_bytes(n, 5, 1, 1, 3) == [2 * n + 2 * dirs, 2 * n + 2 * dirs, n + dirs]
    # 32-bit input, 16-bit intermediate levels, one level per pass
    per = bench.level_pass_bytes(n, 3, 4, 2, 3)
    assert per == [n * (4 + 2) + dirs, n * (2 + 2) + dirs, n * 2 + dirs]


def test_traffic_lookup_dominant_kernel(tmp_path, monkeypatch):
    kernels = {
        "level_pass_u8<true, true, true, false>": {"launches": 30, "fetch_bytes": 100.0, "write_bytes": 50.0},
        "level_pass_u8<true, true, true, true>": {"launches": 5, "fetch_bytes": 100.0, "write_bytes": 20.0},
        "stats_prep_u8<false>": {"launches": 5, "fetch_bytes": 100.0, "write_bytes": 0.0},
    }
    doc = {"w": {"source_sha256": bench.source_sha(), "kernels": kernels, "traffic_bytes_per_launch": 145.7}}
    path = tmp_path / "t.json"
    path.write_text(json.dumps(doc))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    assert bench.traffic_per_launch("w") == 145.7
    assert bench.traffic_per_launch("w", dominant=True) == 150.0
    assert bench.traffic_per_launch("other") is None
    # counters taken on other kernel sources are not used
    doc["w"]["source_sha256"] = "0" * 64
    path.write_text(json.dumps(doc))
    assert bench.traffic_per_launch("w", dominant=True) is None
