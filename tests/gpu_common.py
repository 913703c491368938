"""Shared helpers of the GPU parity tests: library contexts and oracle parameters
for the named rings, and conversion between torch device tensors and numpy."""
import math
import sys

import numpy as np

import workloads as W


def ring_args(ring_name):
    r = W.RINGS[ring_name]
    return dict(log_n=int(math.log2(r.n)), p=r.p, L=r.L, q_bits=r.q_bits, K=r.K, p_bits=r.p_bits)


def oracle_params(ring_name):
    from oracle.params import make_params
    r = W.RINGS[ring_name]
    return make_params(r.n, r.p, r.L, r.q_bits, r.K, r.p_bits)


_CTX = {}


def context(ring_name):
    from paper_2408_17063_amd import hc
    if ring_name not in _CTX:
        _CTX[ring_name] = hc.Context(**ring_args(ring_name))
    return _CTX[ring_name]


def to_dev(arr):
    import torch
    a = np.ascontiguousarray(arr, dtype=np.uint64).view(np.int64)
    return torch.from_numpy(a.copy()).cuda()


def to_host(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint64)


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
