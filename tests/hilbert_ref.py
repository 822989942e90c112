"""Hilbert index of level-21 cells from their Morton keys, in numpy, for the
tests: the transposition algorithm of J. Skilling, "Programming the Hilbert
curve", AIP Conf. Proc. 707, 381 (2004), bit by bit on whole arrays."""
import numpy as np


def hilbert_from_morton(keys):
    keys = keys.astype(np.uint64)
    one = np.uint64(1)
    n = keys.size
    X = [np.zeros(n, np.uint64) for _ in range(3)]
    for b in range(21):
        for i in range(3):
            X[i] |= ((keys >> np.uint64(3 * b + 2 - i)) & one) << np.uint64(b)
    q = 1 << 20
    while q > 1:
        Q, P = np.uint64(q), np.uint64(q - 1)
        for i in range(3):
            hit = (X[i] & Q) != 0
            swap = np.where(hit, np.uint64(0), (X[0] ^ X[i]) & P)
            X[0] = np.where(hit, X[0] ^ P, X[0] ^ swap)
            if i:
                X[i] = X[i] ^ swap
        q >>= 1
    X[1] ^= X[0]
    X[2] ^= X[1]
    t = np.zeros(n, np.uint64)
    q = 1 << 20
    while q > 1:
        t = np.where((X[2] & np.uint64(q)) != 0, t ^ np.uint64(q - 1), t)
        q >>= 1
    h = np.zeros(n, np.uint64)
    for b in range(21):
        for i in range(3):
            h |= (((X[i] ^ t) >> np.uint64(b)) & one) << np.uint64(3 * b + 2 - i)
    return h
