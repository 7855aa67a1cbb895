"""Helpers shared by the GPU tests: device buffers of 32-bit words via torch."""
import numpy as np

import synth


def dev_words(arr):
    """numpy uint32 array -> int32 CUDA tensor with the same bytes."""
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint32)
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def host_words(t):
    return t.cpu().numpy().view(np.uint32)


def ints_to_dev(values):
    return dev_words(synth.ints_to_limbs(values))


def dev_to_ints(t):
    return synth.limbs_to_ints(host_words(t).reshape(-1, 8))


def g1_points_to_words(points):
    """Affine oracle points (None = infinity) -> [n, 16] uint32 canonical words."""
    vals = []
    for p in points:
        vals += [0, 0] if p is None else [p[0], p[1]]
    return synth.ints_to_limbs(vals).reshape(-1, 16)


def g2_points_to_words(points):
    vals = []
    for p in points:
        vals += [0, 0, 0, 0] if p is None else [p[0][0], p[0][1], p[1][0], p[1][1]]
    return synth.ints_to_limbs(vals).reshape(-1, 32)


def words_to_g1_points(words):
    ints = synth.limbs_to_ints(np.asarray(words, dtype=np.uint32).reshape(-1, 8))
    out = []
    for k in range(0, len(ints), 2):
        x, y = ints[k], ints[k + 1]
        out.append(None if x == 0 and y == 0 else (x, y))
    return out


def words_to_g2_points(words):
    ints = synth.limbs_to_ints(np.asarray(words, dtype=np.uint32).reshape(-1, 8))
    out = []
    for k in range(0, len(ints), 4):
        v = ints[k:k + 4]
        out.append(None if not any(v) else ((v[0], v[1]), (v[2], v[3])))
    return out
