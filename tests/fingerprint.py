"""Order-independent fingerprint of a symmetric CSR's edge set, in numpy.

Each undirected edge {i, j}, i < j, is packed as i * 2^32 + j and hashed with
SplitMix64's finaliser (Steele, Lea and Flood, OOPSLA 2014); the fingerprint
is the wrapping sum and the xor of the hashes.  Written apart from the
oracle's C version so that each checks the other."""
import hashlib

import numpy as np

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def csr_fingerprint(row_ptr, col):
    """(sum, xor) over the entries with col > row, as Python ints."""
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr))
    up = col > src
    h = mix64((src[up].astype(np.uint64) << np.uint64(32)) | col[up].astype(np.uint64))
    s = int(np.sum(h, dtype=np.uint64)) if h.size else 0
    x = int(np.bitwise_xor.reduce(h)) if h.size else 0
    return s, x


def degree_sha256(deg):
    return hashlib.sha256(np.ascontiguousarray(deg, dtype=np.int32).tobytes()).hexdigest()
