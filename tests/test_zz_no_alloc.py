"""The allocation-free adaptive-exponent encode (cmg_abfp_encode_noalloc)
against the encode with a caller workspace (cmg_abfp_encode), through the C
ABI: two calls in a row on the static workspace, the second with a smaller
input, each equal bit for bit to the workspace version (codes, kept
blocks, their count) and decoding to the same values."""
import pytest
import torch

import synthetic as S

pytestmark = pytest.mark.gpu


def test_noalloc_encode_matches_workspace_encode(gpu_lib):
    import paper_2511_19036_amd as cmg
    for n, kind, bits, f64 in ((3_000_017, "rising", 16, True), (70_001, "binades", 12, False)):
        x = torch.from_numpy(S.exponent_mix(n, kind, seed=n % 97)).cuda()
        if not f64:
            x = x.float()
        ref = cmg.abfp_encode(x, bits)
        codes = torch.full_like(ref[0], 0x5A)           # stale contents must not matter
        starts = torch.full_like(ref[1], -7)
        exps = torch.full_like(ref[2], 99)
        nblocks = torch.full_like(ref[3], -9)
        cmg.abfp_encode_noalloc(x, bits, codes, starts, exps, nblocks)
        torch.cuda.synchronize()
        nb = int(ref[3].item())
        assert nb >= 1 and int(nblocks.item()) == nb, (n, nb)
        nbytes = int(cmg.load().cmg_abfp_code_bytes(n, bits))
        assert torch.equal(codes[:nbytes], ref[0][:nbytes]), n
        assert torch.equal(starts[:nb], ref[1][:nb]) and torch.equal(exps[:nb], ref[2][:nb]), n
        assert torch.equal(cmg.abfp_decode(codes, starts, exps, nblocks, n, bits),
                           cmg.abfp_decode(*ref, n, bits)), n
