"""The streaming kernel behind the benchmark's HBM ceiling copies (or adds)
exactly, in every access form and on grids that do not divide the array:
its GB/s only mean something if it moved every byte once."""

import pytest
import torch

from gpuhelp import note

pytestmark = pytest.mark.gpu

import paper_2310_01882_amd as ms  # noqa: E402


@pytest.mark.parametrize("form", [0, 1, 2, 3])
@pytest.mark.parametrize("two", [False, True])
def test_stream_probe_moves_every_element_once(form, two):
    g = torch.Generator().manual_seed(7 + form)
    for n in (2, 1000, 2 * (1 << 20) + 6):
        for blocks in (1, 7, 512):
            note(f"case: stream probe form={form} two={two} n={n} blocks={blocks}")
            a = torch.rand(n, generator=g, dtype=torch.float64).cuda()
            b = torch.rand(n, generator=g, dtype=torch.float64).cuda() if two else None
            out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
            ms.stream_probe(a, out, b, blocks=blocks, form=form)
            torch.cuda.synchronize()
            assert torch.equal(out, a + b if two else a)


def test_stream_probe_rejects_bad_arguments():
    a = torch.zeros(7, dtype=torch.float64, device="cuda")
    with pytest.raises(ms.MsError):
        ms.stream_probe(a, torch.zeros_like(a))  # odd length
    a = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(ms.MsError):
        ms.stream_probe(a, torch.zeros_like(a), form=4)
    with pytest.raises(ms.MsError):
        ms.stream_probe(a, a)  # out overlaps the input
