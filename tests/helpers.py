"""Shared helpers of the GPU parity tests (no exchange arithmetic here)."""
import numpy as np

PERMS = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
         (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]


def _pack_img(n):
    return (n[..., 0] + 16) * 1024 + (n[..., 1] + 16) * 32 + (n[..., 2] + 16)


def canonical_keys(inst):
    """inst: (n, 4, 4) int64 = [shell, n1, n2, n3] of the four shell
    instances (bra1, bra2, ket1, ket2).  Returns an (n, 2) int64 key of the
    orbit under the 8 index orders of the permutation relations, each
    translated so that its first shell sits in the home cell."""
    inst = np.asarray(inst, dtype=np.int64)
    k1s, k2s = [], []
    for p in PERMS:
        a = inst[:, list(p), :].copy()
        a[:, :, 1:] -= a[:, 0:1, 1:]
        k1 = ((a[:, 0, 0] * 4096 + a[:, 1, 0]) * 32768 + _pack_img(a[:, 1, 1:])) * 4096 + a[:, 2, 0]
        k2 = (_pack_img(a[:, 2, 1:]) * 4096 + a[:, 3, 0]) * 32768 + _pack_img(a[:, 3, 1:])
        k1s.append(k1)
        k2s.append(k2)
    k1 = np.stack(k1s, axis=1)
    k2 = np.stack(k2s, axis=1)
    m1 = k1.min(axis=1)
    m2 = np.where(k1 == m1[:, None], k2, np.iinfo(np.int64).max).min(axis=1)
    return np.stack([m1, m2], axis=1)


def gpu_quartet_instances(quartets, pairs):
    """GPU list (n,5: bra, ket, G) + pair table (A, B, n(3), class) -> (n,4,4)."""
    q = np.asarray(quartets, dtype=np.int64)
    pr = np.asarray(pairs, dtype=np.int64)
    b = pr[q[:, 0]]
    k = pr[q[:, 1]]
    G = q[:, 2:5]
    inst = np.zeros((len(q), 4, 4), dtype=np.int64)
    inst[:, 0, 0] = b[:, 0]
    inst[:, 1, 0] = b[:, 1]
    inst[:, 1, 1:] = b[:, 2:5]
    inst[:, 2, 0] = k[:, 0]
    inst[:, 2, 1:] = G
    inst[:, 3, 0] = k[:, 1]
    inst[:, 3, 1:] = G + k[:, 2:5]
    return inst


def oracle_quartet_instances(rows):
    """Oracle rows (I, J, N(3), K, L, M(3), G(3)) -> (n,4,4) with H = G + M."""
    r = np.asarray(rows, dtype=np.int64)
    inst = np.zeros((len(r), 4, 4), dtype=np.int64)
    inst[:, 0, 0] = r[:, 0]
    inst[:, 1, 0] = r[:, 1]
    inst[:, 1, 1:] = r[:, 2:5]
    inst[:, 2, 0] = r[:, 5]
    inst[:, 2, 1:] = r[:, 10:13]
    inst[:, 3, 0] = r[:, 6]
    inst[:, 3, 1:] = r[:, 10:13] + r[:, 7:10]
    return inst


def key_set(keys):
    return set(map(tuple, np.asarray(keys).tolist()))
