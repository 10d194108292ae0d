"""Helpers of the GPU tests: run the C-ABI path and the oracle on the same bytes."""
import numpy as np
import pytest
import torch

import oracle


def device():
    if not torch.cuda.is_available():
        pytest.skip("needs a HIP device")
    return torch.device("cuda:0")


def u32(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy().view(np.uint32)


def gpu_tree(f: np.ndarray, dev):
    import paper_2301_10838_amd.mt as mt

    ft = torch.from_numpy(np.ascontiguousarray(f)).to(dev)
    ws = mt.alloc_workspace(mt.workspace_bytes(f.shape), dev)
    T = mt.mt_build(ft, workspace=ws)
    b, d, bv, dv, nroots = mt.mt_persistence_pairs(ft, T, workspace=ws)
    torch.cuda.synchronize()
    return u32(T).reshape(-1, 2), (u32(b), u32(d), bv.cpu().numpy(), dv.cpu().numpy(), nroots)


def assert_matches_oracle(f: np.ndarray, T, prs, what=""):
    T_ref = oracle.merge_tree(f)
    rb, rd, rbv, rdv, rroots = oracle.pairs(f, T_ref)
    if not np.array_equal(T, T_ref):
        bad = np.nonzero(np.any(T != T_ref, axis=1))[0]
        raise AssertionError(f"{what}: {bad.size} triplets differ, first at u={bad[0]}: gpu {T[bad[0]].tolist()} "
                             f"oracle {T_ref[bad[0]].tolist()}")
    b, d, bv, dv, nroots = prs
    assert np.array_equal(b, rb), what
    assert np.array_equal(d, rd), what
    # values are bit copies of the float32 field
    flat = np.asarray(f, np.float32).reshape(-1)
    assert np.array_equal(bv.view(np.uint32), flat[rb].view(np.uint32)), what
    assert np.array_equal(dv.view(np.uint32), flat[rd].view(np.uint32)), what
    assert nroots == rroots, what
