"""Host-side pieces of bench.py: the traffic figures are taken from the
committed counter summary only while the kernel sources and launch
parameters match."""
import bench


def _write(tmp_path, sha, launch="0.5,64", line="traffic_bytes neighbours: 1234"):
    p = tmp_path / "traffic.md"
    p.write_text(f"```\nsource_sha256: {sha}\nlaunch: {launch}\n{line}\n```\n")
    return str(p)


def _sources_sha():
    return bench.kernel_code_digest()


def test_code_digest_ignores_comments_and_white_space(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    py = tmp_path / "b.py"
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ["k.hip", "b.py"])

    def digest(hip, pyt):
        src.write_text(hip)
        py.write_text(pyt)
        return bench.kernel_code_digest()
    d0 = digest("int f(int a) { return a + 1; }\n", "X = 1\n")
    assert digest("// a note\nint f(int a)\n{\n  return a + 1;  /* the next */\n}\n",
                  "X = 1  # one\n") == d0
    assert digest("int f(int a) { return a + 2; }\n", "X = 1\n") != d0
    assert digest("int f(int a) { return a + 1; }\n", "X = 2\n") != d0


def test_traffic_only_for_matching_sources_and_launch(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _write(tmp_path, _sources_sha()))
    assert bench.measured_traffic("neighbours", 0.5, 64) == 1234
    assert bench.measured_traffic("tracklets", 0.5, 64) is None
    assert bench.measured_traffic("neighbours", 1.0, 64) is None
    assert bench.measured_traffic("neighbours", 0.5, 128) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", _write(tmp_path, "0" * 64))
    assert bench.measured_traffic("neighbours", 0.5, 64) is None
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(tmp_path / "missing.md"))
    assert bench.measured_traffic("neighbours", 0.5, 64) is None


def test_traffic_block_of_the_matching_launch(tmp_path, monkeypatch):
    p = tmp_path / "traffic.md"
    p.write_text(f"```\nsource_sha256: {_sources_sha()}\n"
                 "launch: 1.0,64\ntraffic_bytes neighbours: 11\ntraffic_bytes tracklets: 12\n"
                 "launch: 0.5,64\ntraffic_bytes neighbours: 21\n```\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILE", str(p))
    assert bench.measured_traffic("neighbours", 1.0, 64) == 11
    assert bench.measured_traffic("tracklets", 1.0, 64) == 12
    assert bench.measured_traffic("neighbours", 0.5, 64) == 21
    # a kernel missing from its own block is not taken from another block
    assert bench.measured_traffic("tracklets", 0.5, 64) is None
    assert bench.measured_traffic("neighbours", 2.0, 64) is None


def test_committed_summaries_parse():
    # the committed counter summaries carry blocks for the usual launch
    # configuration (values present whenever the sources still match)
    for f in (bench.TRAFFIC_PROFILE,):
        text = open(f).read()
        assert "source_sha256: " in text and "launch: 1.0,64" in text


def test_differently_assigned_counts():
    import numpy as np
    a = {"clu2trk": np.array([0, 0, 0, 1, 1, -1, 2, 2])}
    b = {"clu2trk": np.array([5, 5, 4, 3, 3, -1, -1, 7])}
    # track 0 -> 5 (two of three), so cluster 2 on track 4 differs; cluster 6
    # is unassigned in b only
    assert bench.differently_assigned(a, b, 8) == {"clusters": 2, "fraction": 0.25}
    assert bench.differently_assigned(a, a, 8)["clusters"] == 0
