"""The plain streaming kernels of the roofline's achievable ceiling (ctu_stream_probe) compute
what they claim, so that the bandwidth they report belongs to real reads and writes: the read
kernel's block sums add up to the array's sum, copy copies, add adds, and the 5:1 combine sums
five arrays, on sizes that leave a ragged last block."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 1000, 1024, 262147])
def test_stream_probe_kernels_compute_what_they_claim(n):
    import torch
    from paper_1410_4194_amd import ctu
    print(f"[gpu-test] stream probe n={n}", flush=True)
    g = torch.Generator(device="cpu").manual_seed(n)
    a_h = torch.rand(5 * n, dtype=torch.float64, generator=g)
    b_h = torch.rand(n, dtype=torch.float64, generator=g)
    a = a_h.cuda()
    b = b_h.cuda()
    nb = ctu.stream_probe_blocks(5 * n)
    c = torch.full((max(5 * n, nb),), float("nan"), dtype=torch.float64, device="cuda")
    ctu.stream_probe(ctu.STREAM_READ, a, None, c, 5 * n)
    torch.cuda.synchronize()
    parts = c[:nb].cpu().numpy()
    assert np.isfinite(parts).all()
    assert abs(parts.sum() - a_h.sum().item()) <= 1e-12 * a_h.abs().sum().item()
    for kind, ref in ((ctu.STREAM_COPY, a_h[:n]), (ctu.STREAM_ADD, a_h[:n] + b_h),
                      (ctu.STREAM_COMBINE5, a_h.view(5, n).sum(0))):
        c.fill_(float("nan"))
        ctu.stream_probe(kind, a, b if kind == ctu.STREAM_ADD else None, c, n)
        torch.cuda.synchronize()
        got = c[:n].cpu()
        if kind == ctu.STREAM_COMBINE5:
            assert torch.allclose(got, ref, rtol=1e-15, atol=0.0)
        else:
            assert torch.equal(got, ref)
        assert torch.isnan(c[n:]).all()  # nothing written past the end
