"""Row layouts of the tables the shading kernels gather from (no torch).

A texel row is read whole for every path vertex that names it, at random.
Every miss costs whole 128-byte lines, so a row should touch no more lines
than its length needs: rows of at most 32 floats get a power-of-two stride
(they then never cross a line boundary), longer rows a multiple of 32 floats.
"""


def blocks(k: int) -> int:
    """Number of RGB-style passes B for a k-channel code (k padded to 3B)."""
    return (k + 2) // 3


def latent_width(k: int) -> int:
    """Floats per latent row in the blocked RGBx layout (4 per block)."""
    return 4 * blocks(k)


def line_stride(width: int) -> int:
    """Row stride in floats for rows of `width` floats that are gathered at
    random: 31 samples -> 32, 81 -> 96, k = 6 codes (8 floats) -> 8, k = 9
    codes (12 floats) -> 16, k = 48 (64 floats) -> 64."""
    w = 4 * ((width + 3) // 4)
    if w <= 32:
        p = 4
        while p < w:
            p *= 2
        return p
    return 32 * ((w + 31) // 32)
