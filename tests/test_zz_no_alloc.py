"""The allocation-free forward pass of the surrogate network
(md_mlp_forward_noalloc, intermediates in the library's static device
buffer) against md_mlp_forward on the same network and inputs: bitwise equal
outputs on two calls in a row, the second with a smaller ragged batch (the
buffer still holds the first call's larger contents), and a batch beyond the
buffer refused on the host."""
import numpy as np
import pytest

from paper_2606_08039_amd import md

pytestmark = pytest.mark.gpu


def _network(rng):
    parts = []
    for sh in md.MLP_SHAPES:
        parts.append(rng.normal(size=sh) * (np.sqrt(2.0 / sh[1]) if len(sh) == 2 else 0.1))
    norm = np.concatenate([rng.normal(size=64) * 0.3, rng.uniform(0.5, 3.0, size=64),
                           rng.normal(size=6) * 0.01, rng.uniform(0.01, 0.1, size=6)])
    return md.mlp_flatten(parts), norm.astype(np.float32)


def test_noalloc_forward_equals_forward_on_two_calls():
    import torch
    rng = np.random.default_rng(2024)
    flat, norm = _network(rng)
    B_max = md.MD_MLP_NOALLOC_MAX_BATCH
    m = md.md_mlp_create(B_max)
    try:
        md.md_mlp_set_params(m, flat)
        md.md_mlp_set_norm(m, norm)
        for B in (B_max, 1001):
            print("md_mlp_forward_noalloc B=%d" % B, flush=True)
            X = torch.from_numpy(rng.normal(size=(B, 64)).astype(np.float32)).cuda()
            ref = torch.full((B, 6), float("nan"), device="cuda")
            got = torch.full((B, 6), float("nan"), device="cuda")
            md.md_mlp_forward(m, X, Y=ref)
            md.md_mlp_forward_noalloc(m, X, got)
            torch.cuda.synchronize()
            r, g = ref.cpu().numpy(), got.cpu().numpy()
            assert np.isfinite(r).all()
            np.testing.assert_array_equal(g, r, err_msg="batch %d" % B)
        with pytest.raises(md.MdError) as ei:
            X = torch.zeros((B_max + 1, 64), device="cuda")
            md.md_mlp_forward_noalloc(m, X, torch.zeros((B_max + 1, 6), device="cuda"))
        assert ei.value.status == md.MD_E_INVALID_ARG
        assert "exceeds" in md.lib().md_mlp_last_error(m).decode()
    finally:
        md.md_mlp_destroy(m)
