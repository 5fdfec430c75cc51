"""Oracle for the restricted tune space (test infrastructure only).

Section IV describes the search space as the Cartesian product of the
tunable parameters' value lists, of which many portions are restricted; the
DVFS knobs (section III.C) multiply it further.  The convolution's tunables
are block_size_x, block_size_y, tile_size_x, tile_size_y, use_lds_padding and
read_path.  Restrictions (the kernel's launch limits):

* threads per block  block_size_x * block_size_y <= max_threads
* LDS-staged configs (read_path 0) must fit the per-block LDS limit:
      pitch = ceil4(block_size_x*tile_size_x + fw - 1) + 4*use_lds_padding   (floats)
      rows  = block_size_y*tile_size_y + fh - 1
      bytes = 4 * pitch * rows
* direct-read configs (read_path 1) stage nothing, so use_lds_padding = 1 is a
  duplicate of use_lds_padding = 0 and is dropped when ``dedup_direct``.

Order: itertools.product over (bx, by, tx, ty, pad, read_path), last fastest.
"""
import itertools

NAMES = ("block_size_x", "block_size_y", "tile_size_x", "tile_size_y",
         "use_lds_padding", "read_path")


def lds_bytes(bx, by, tx, ty, pad, fh, fw):
    w = bx * tx + fw - 1
    pitch = (w + 3) // 4 * 4 + 4 * pad
    return 4 * pitch * (by * ty + fh - 1)


def enumerate_space(values, fh, fw, max_threads=1024, lds_limit=65536, dedup_direct=True):
    lists = [values[n] for n in NAMES]
    out = []
    for bx, by, tx, ty, pad, rp in itertools.product(*lists):
        if bx * by > max_threads:
            continue
        if rp == 0 and lds_bytes(bx, by, tx, ty, pad, fh, fw) > lds_limit:
            continue
        if rp == 1 and pad != 0 and dedup_direct:
            continue
        out.append((bx, by, tx, ty, pad, rp))
    return out
