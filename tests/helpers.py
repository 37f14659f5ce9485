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


def orbit_members(rows):
    """Distinct ordered quartets of the orbits of the given ordered quartets
    under the 8 index orders of the permutation relations, each translated
    so that its first shell sits in the home cell.  rows: (n, 13) oracle
    rows (I, J, N(3), K, L, M(3), G(3)), L at G + M.  Returns (m, 13)."""
    inst = oracle_quartet_instances(rows)
    out = set()
    for q in inst:
        for p in PERMS:
            a = q[list(p)].copy()
            a[:, 1:] -= a[0, 1:]
            I, J, K, L = a[:, 0]
            N, G, H = a[1, 1:], a[2, 1:], a[3, 1:]
            out.add((int(I), int(J), *map(int, N), int(K), int(L), *map(int, H - G), *map(int, G)))
    return np.array(sorted(out), dtype=np.int64).reshape(-1, 13)


def gpu_rows(quartets, pairs):
    """GPU list (n,5: bra, ket, G) + pair table -> oracle rows (n, 13)."""
    inst = gpu_quartet_instances(quartets, pairs)
    r = np.zeros((len(inst), 13), dtype=np.int64)
    r[:, 0] = inst[:, 0, 0]
    r[:, 1] = inst[:, 1, 0]
    r[:, 2:5] = inst[:, 1, 1:]
    r[:, 5] = inst[:, 2, 0]
    r[:, 6] = inst[:, 3, 0]
    r[:, 7:10] = inst[:, 3, 1:] - inst[:, 2, 1:]
    r[:, 10:13] = inst[:, 2, 1:]
    return r


def to_gpu_quartets(rows, pairs, pair_class_of):
    """One member of each ordered quartet's orbit in the device encoding
    (bra pair | ket pair << 24 | translation << 48): the member whose bra
    and ket pairs appear in the unique-pair table (A, B, n) in that
    orientation, with class(bra) >= class(ket).  Returns uint64 array."""
    index = {(int(a), int(b), int(n1), int(n2), int(n3)): i for i, (a, b, n1, n2, n3, _) in enumerate(pairs)}
    out = []
    for q in oracle_quartet_instances(rows):
        found = None
        for p in PERMS:
            a = q[list(p)].copy()
            a[:, 1:] -= a[0, 1:]
            bra = index.get((int(a[0, 0]), int(a[1, 0]), *map(int, a[1, 1:])))
            G = a[2, 1:]
            ket = index.get((int(a[2, 0]), int(a[3, 0]), *map(int, a[3, 1:] - G)))
            if bra is None or ket is None or pair_class_of[bra] < pair_class_of[ket]:
                continue
            if np.any(np.abs(G) > 15):
                continue
            g = int((G[0] + 16) | ((G[1] + 16) << 5) | ((G[2] + 16) << 10))
            found = np.uint64(bra) | (np.uint64(ket) << np.uint64(24)) | (np.uint64(g) << np.uint64(48))
            break
        assert found is not None, "no member of the orbit in device orientation"
        out.append(found)
    return np.array(out, dtype=np.uint64)
