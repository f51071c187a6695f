"""The packed-chunk rules of the batched 2D passes (csrc/wt_pack.hpp), on the CPU: for
lines of W interfaces (W = points + 1 along the pass), every chunk respects its
interface and staging limits, every cell is finished by exactly one chunk, and every
stencil row of every interface stages the point the stencil needs.  The GPU kernel
reads its staging offsets from the same functions, so a table that passes here cannot
make it read outside its staged rows."""
import pytest

from tests import host_kernel as HK

# (interface rows per chunk, staged rows per chunk) as the kernels use them, and two
# other limits (a longer chunk, and a tight staging limit)
_, _QT, _ROWS = HK.pack_limits()
CONFIGS = [(_QT, _ROWS), (256, 296), (32, 40)]
WIDTHS = [7, 8, 9, 16, 31, 32, 33, 40, 57, 63, 64, 65, 97, 128, 200, 257]
LINES = [1, 2, 3, 5, 8, 13, 40]


@pytest.mark.parametrize("qt,rmax", CONFIGS)
def test_packed_chunks_cover_every_cell_once_and_stage_every_stencil(qt, rmax):
    for W in WIDTHS:
        for nl in LINES:
            Q = W * nl
            chunks = HK.pack_chunks(W, nl, qt, rmax)
            finished = [0] * Q
            seen = [False] * Q
            prev_end = None
            for q0, nq in chunks:
                assert 2 <= nq <= qt and q0 >= 0 and q0 + nq <= Q, (W, nl, q0, nq)
                rows = HK.pack_rows(q0, nq, W)
                assert rows <= rmax, (W, nl, q0, nq, rows)
                # consecutive chunks overlap by one interface, except after a line end
                if prev_end is not None:
                    assert q0 == (prev_end + 1 if prev_end % W == W - 1 else prev_end), (W, nl)
                prev_end = q0 + nq - 1
                staged = [HK.pack_point(q0, r, W) for r in range(rows)]
                for q in range(q0, q0 + nq):
                    seen[q] = True
                    line, i = divmod(q, W)
                    base = HK.pack_base(q0, q, W)
                    assert 0 <= base and base + 5 < rows, (W, nl, q0, q)
                    for k in range(6):
                        assert staged[base + k] == (line, i - 3 + k), (W, nl, q0, q, k)
                    if q < q0 + nq - 1 and i < W - 1:
                        finished[q] += 1
            assert prev_end == Q - 1
            assert all(seen)
            for q in range(Q):
                assert finished[q] == (1 if q % W < W - 1 else 0), (W, nl, q)


def test_packed_chunks_fill_the_threads_on_the_benchmark_sizes():
    """On lines of 32 to 96 points the chunks use at least 95% of their interface rows,
    against 72% of the slots for the fixed 8 x 31 tiles (the lines' own raggedness, groups
    of 8 rows or columns, comes on top in both)."""
    lanes, qt, rmax = HK.pack_limits()
    assert lanes * qt == 256
    used = total = 0
    for n in range(32, 97):
        chunks = HK.pack_chunks(n + 1, 8, qt, rmax)
        used += sum(nq for _, nq in chunks)
        total += qt * len(chunks)
    assert used / total >= 0.95, used / total
