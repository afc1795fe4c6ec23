"""Helpers shared by the GPU parity tests (host <-> device marshalling and the
oracle comparisons)."""
import numpy as np

import oracle as O


def to_dev(a):
    import torch
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        t = torch.from_numpy(a.view(np.int64))
    elif a.dtype == np.uint32:
        t = torch.from_numpy(a.view(np.int32))
    else:
        raise TypeError(a.dtype)
    return t.cuda()


def to_host(t, dtype):
    a = t.cpu().numpy()
    return a.view(dtype)


def assert_semisort_equal(keys, vals, ko, vo, mode=O.HASH_MIX64, ctx=""):
    """GPU output (ko, vo) must be a stable semisort of (keys, vals): same
    canonical form as the oracle's result."""
    rk, rv = O.semisort_equal(keys, vals, mode)
    bad, ck, cv = O.canonicalize_equal(ko, vo, mode)
    assert bad == -1, f"{ctx}: key at position {bad} starts a second run (equal keys not contiguous)"
    if not np.array_equal(ck, rk):
        i = int(np.nonzero(ck != rk)[0][0])
        raise AssertionError(f"{ctx}: keys differ from the oracle at canonical position {i}")
    if not np.array_equal(cv, rv):
        i = int(np.nonzero(cv != rv)[0][0])
        raise AssertionError(f"{ctx}: values differ from the oracle at canonical position {i} (stability or moves)")
