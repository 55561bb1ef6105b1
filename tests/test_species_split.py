"""Host logic of the per-species networks: cutting one-output networks from a
K-output network's public parameter vector (no GPU)."""
import numpy as np

from oracle import ann as oann
from paper_2402_18858_amd import train


def _unpack(params, dims):
    Ws, bs, off = [], [], 0
    for i in range(len(dims) - 1):
        n = dims[i] * dims[i + 1]
        Ws.append(params[off:off + n].reshape(dims[i], dims[i + 1]).astype(np.float64))
        off += n
        bs.append(params[off:off + dims[i + 1]].astype(np.float64))
        off += dims[i + 1]
    return Ws, bs


def test_species_slice_matches_the_oracle_split():
    dims = [9, 20, 12, 7]
    rng = np.random.default_rng(1)
    params = rng.normal(size=sum(dims[i] * dims[i + 1] + dims[i + 1] for i in range(3))).astype(np.float32)
    Ws, bs = _unpack(params, dims)
    ref = oann.species_split(Ws, bs)
    one = dims[:-1] + [1]
    for k in range(dims[-1]):
        v = train.species_slice(params, dims, k)
        assert v.size == sum(one[i] * one[i + 1] + one[i + 1] for i in range(3))
        W, b = _unpack(v, one)
        for a, r in zip(W + b, ref[k][0] + ref[k][1]):
            np.testing.assert_array_equal(a, r)
    # outputs agree with the K-output network's columns
    X = rng.normal(size=(5, 9))
    full, _ = oann.forward(Ws, bs, X, quantize=False)
    nets = [_unpack(train.species_slice(params, dims, k), one) for k in range(dims[-1])]
    np.testing.assert_allclose(oann.species_forward(nets, X, quantize=False), full, rtol=1e-13, atol=1e-15)
