"""Trajectory files and results files on the CPU: the library's reader
accepts what the writer produces and rejects damaged files (no device work),
and the results parser reads the documented record layout."""
import numpy as np
import pytest

import workloads


@pytest.fixture(scope="module")
def dh():
    import paper_1808_01478_amd as dh
    return dh


def frames(n_frames=3, n=50, seed=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return [rng.uniform(0, 10, size=(n, 3)) for _ in range(n_frames)]


def test_open_and_info(dh, tmp_path):
    from paper_1808_01478_amd import trajfile
    p = str(tmp_path / "t.dhtraj")
    box = workloads.ortho_box(10.0, 11.0, 12.0)
    assert trajfile.write_trajectory(p, frames(), 1, [box] * 3) == 3
    with dh.Trajectory(p) as t:
        assert t.info() == {"n_frames": 3, "n_points": 50, "box_type": 1}
    pn = str(tmp_path / "none.dhtraj")
    trajfile.write_trajectory(pn, frames(2, 7), 0)
    with dh.Trajectory(pn) as t:
        assert t.info() == {"n_frames": 2, "n_points": 7, "box_type": 0}


def test_damaged_files_rejected(dh, tmp_path):
    from paper_1808_01478_amd import trajfile
    p = str(tmp_path / "t.dhtraj")
    trajfile.write_trajectory(p, frames(), 0)
    raw = open(p, "rb").read()
    bad = [raw[:-8],                                 # truncated
           raw + b"\0" * 8,                          # trailing bytes
           b"XHTRAJ01" + raw[8:],                    # magic
           raw[:24] + np.int32(7).tobytes() + raw[28:]]   # box type
    for k, b in enumerate(bad):
        q = str(tmp_path / f"bad{k}.dhtraj")
        open(q, "wb").write(b)
        with pytest.raises(dh.DisthistError) as e:
            dh.Trajectory(q)
        assert e.value.code == -1
    with pytest.raises(dh.DisthistError):
        dh.Trajectory(str(tmp_path / "missing.dhtraj"))


def test_results_reader(tmp_path):
    from paper_1808_01478_amd import trajfile
    n_hist, n_bins = 3, 5
    hdr = bytearray(trajfile.RES_HEADER)
    hdr[0:8] = trajfile.RES_MAGIC
    hdr[16:40] = np.array([2, 9, 4], np.int64).tobytes()
    hdr[40:56] = np.array([2, n_bins, 1, 1], np.int32).tobytes()
    hdr[56:64] = np.float64(2.5).tobytes()
    recs = np.arange(2 * (n_hist * n_bins + n_hist + 1), dtype=np.uint64)
    p = tmp_path / "r.dhres"
    p.write_bytes(bytes(hdr) + recs.tobytes() + b"\1\2\3")   # plus a partial record
    info, hist, oor, fr = trajfile.read_results(str(p), n_hist)
    assert info == dict(frame_begin=2, frame_end=9, interval=4, n_species=2, n_bins=5,
                        precision=1, box_type=1, r_max=2.5)
    words = n_hist * n_bins + n_hist + 1
    assert hist.shape == (2, n_hist, n_bins) and oor.shape == (2, n_hist)
    assert hist[1, 0, 0] == words and oor[0, 0] == n_hist * n_bins and list(fr) == [words - 1, 2 * words - 1]
