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
