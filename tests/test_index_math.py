"""Index arithmetic of the staging loops (host check of the kernels' design;
no GPU). The analysis transpose and the FC kernel find the row of a staged
element e as (e + 1/2) times the single-precision reciprocal of the row length,
truncated, instead of an integer division; this is exact only over the ranges
the kernels use, which these tests cover exhaustively in IEEE single precision
(the same operations the device code performs: a correctly rounded 1/w, an
exact e + 1/2, one rounded product). Also the coverage of the analysis window
by the Welch segments, on which the Up/Down kernel's min and max rely."""
import numpy as np
import pytest


def reciprocal_rows(e, w):
    inv = np.float32(1.0) / np.float32(w)
    q = (e.astype(np.float32) + np.float32(0.5)) * inv
    assert q.dtype == np.float32
    return np.trunc(q).astype(np.int64)


def test_transpose_rows_exact():
    """Transpose: tiles of at most 64 x 128 elements (e < 8192), row lengths
    kw = 1..128 (the regions of one chunk)."""
    e = np.arange(64 * 128, dtype=np.int64)
    for kw in range(1, 129):
        np.testing.assert_array_equal(reciprocal_rows(e, kw), e // kw, err_msg=f"kw={kw}")


def test_fc_stage_rows_exact():
    """FC staging: chunks of 4096 doubles (e < 4096), padded row lengths
    npad = 4, 8, ..., 1024 (up to 1024 regions)."""
    e = np.arange(4096, dtype=np.int64)
    for npad in range(4, 1025, 4):
        np.testing.assert_array_equal(reciprocal_rows(e, npad), e // npad, err_msg=f"npad={npad}")


@pytest.mark.parametrize("kw", [3, 5, 7, 68, 127])
def test_transpose_walk_covers_tile_once(kw):
    """Every element of a tile (rows x kw) is staged by exactly one thread
    (thread t takes e = t + 256 j), and every LDS slot the write-back reads
    is filled, including a ragged last tile of the window."""
    for rows in (64, 17, 1):
        ne = rows * kw
        seen = np.zeros((64, 129), np.int64)
        for t in range(256):
            for j in range(64 * 128 // 256):
                e = t + 256 * j
                if e < ne:
                    r = int(reciprocal_rows(np.array([e]), kw)[0])
                    seen[r, e - r * kw] += 1
        assert (seen[:rows, :kw] == 1).all()
        assert seen.sum() == ne


def test_welch_segments_cover_the_window():
    """The Up/Down kernel takes each region's min and max from the Welch
    kernel's segment pass, so the segments (length L, hop L/2, (Na - L)/hop + 1
    of them, as the host computes them) must cover the window [0, Na) exactly
    for every window and segment length the analysis accepts (powers of two,
    16 <= L <= min(Na, 8192), Na <= 16384)."""
    for lna in range(4, 15):
        Na = 1 << lna
        for lL in range(4, 14):
            L = 1 << lL
            if L > Na:
                continue
            hop = L // 2
            n_seg = (Na - L) // hop + 1
            covered = np.zeros(Na, bool)
            for sg in range(n_seg):
                covered[sg * hop:sg * hop + L] = True
            assert covered.all() and (n_seg - 1) * hop + L == Na, (Na, L)
