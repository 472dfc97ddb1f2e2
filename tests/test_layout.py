"""Row strides of gathered tables: every row touches the fewest 128-byte lines
its length allows (rows start at a 128-byte aligned base)."""

from paper_2602_18741_amd.layout import blocks, latent_width, line_stride


def _lines(start_byte, nbytes):
    return (start_byte + nbytes - 1) // 128 - start_byte // 128 + 1


def test_line_stride_minimises_lines_per_row():
    for w in range(1, 161):
        s = line_stride(w)
        assert s >= w and s % 4 == 0
        need = -(-4 * w // 128)          # lines a row of w floats needs at least
        for i in range(256):
            assert _lines(4 * s * i, 4 * w) == need, (w, s, i)


def test_line_stride_overhead_and_examples():
    for w in range(1, 161):
        s = line_stride(w)
        assert s < 2 * max(w, 4) if w <= 32 else s < w + 32
    assert [line_stride(w) for w in (31, 81, 128)] == [32, 96, 128]
    assert [line_stride(latent_width(k)) for k in (3, 6, 9, 48)] == [4, 8, 16, 64]
    assert [blocks(k) for k in (1, 3, 4, 6, 9, 48)] == [1, 1, 2, 2, 3, 16]
