"""Test helpers: convert block data in the library's documented panel layout into the
oracle's dense-tensor MPS (input/output marshalling only, no method arithmetic)."""
import numpy as np

import synth
from oracle import mps as om


def blocks_to_oracle(bonds, data):
    L = len(bonds) - 1
    tensors, labels = [], []
    for i in range(L + 1):
        lab = []
        for nu, nd, d in bonds[i]:
            lab += [(nu, nd)] * d
        labels.append(np.array(lab, dtype=np.int64).reshape(-1, 2))
    off = 0
    for i in range(L):
        left = [((a, b), d) for a, b, d in bonds[i]]
        right = [((a, b), d) for a, b, d in bonds[i + 1]]
        offs, widths, blocks, size = synth._panel_layout(left, right)
        lo = np.cumsum([0] + [d for _, d in left])
        ro = np.cumsum([0] + [d for _, d in right])
        A = np.zeros((lo[-1], 4, ro[-1]), dtype=np.complex128)
        site = data[off:off + size]
        for (s, n), (t, col) in blocks.items():
            ds, dt = left[s][1], right[t][1]
            panel = site[offs[s]:offs[s] + ds * widths[s]].reshape(ds, widths[s])
            A[lo[s]:lo[s] + ds, n, ro[t]:ro[t] + dt] = panel[:, col:col + dt]
        tensors.append(A)
        off += size
    assert off == len(data)
    return om.MPS(tensors, labels)


def lib_to_oracle(m):
    return blocks_to_oracle(m.sectors(), m.get_blocks())


def dense(m):
    """Dense vector of a library state through the oracle's own contraction."""
    return om.to_full(lib_to_oracle(m))


def two_site_index(blocks, bonds, c):
    """For the two-site tensor at bond (c, c+1) in the layout table of tdmps_heff_layout,
    the dense index (a, s1 * 4 + s2, b) of every element, in layout order: returns
    (flat layout offsets, flat dense indices into an array of shape (D_c, 16, D_{c+2}))."""
    lo, ro = {}, {}
    acc = 0
    for nu, nd, d in bonds[c]:
        lo[(nu, nd)] = acc
        acc += d
    Dl = acc
    acc = 0
    for nu, nd, d in bonds[c + 2]:
        ro[(nu, nd)] = acc
        acc += d
    Dr = acc
    offs, idx = [], []
    for row in blocks:
        nu, nd, n1, n2, Da, Db = [int(v) for v in row[:6]]
        off = (int(row[6]) | (int(row[7]) << 31)) // 2
        ld = int(row[8])
        qb = (nu + (n1 & 1) + (n2 & 1), nd + (n1 >> 1) + (n2 >> 1))
        a = lo[(nu, nd)] + np.arange(Da)
        b = ro[qb] + np.arange(Db)
        offs.append((off + np.arange(Da)[:, None] * ld + np.arange(Db)[None, :]).reshape(-1))
        idx.append(((a[:, None] * 16 + (n1 * 4 + n2)) * Dr + b[None, :]).reshape(-1))
    return np.concatenate(offs), np.concatenate(idx), (Dl, 16, Dr)
