"""dg_triad, the bandwidth probe of the measurements (GPU): every element of
out = a + s b, at a length that leaves a partial last pass of the grid, and
the alignment rule."""
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("n", [2, 1000, (1 << 20) + 6, 3 * (1 << 21) + 2])
def test_triad_is_exact_on_integers(n):
    from paper_2511_05233_amd import lsbdg
    g = torch.Generator(device="cuda:0").manual_seed(n)
    a = torch.randint(-2 ** 20, 2 ** 20, (n,), generator=g, device="cuda:0").double()
    b = torch.randint(-2 ** 20, 2 ** 20, (n,), generator=g, device="cuda:0").double()
    out = torch.full_like(a, float("nan"))
    lsbdg.triad(out, a, b, 0.5)
    torch.cuda.synchronize()
    assert torch.equal(out, a + 0.5 * b)


def test_triad_refuses_odd_lengths_and_misaligned_arrays():
    from paper_2511_05233_amd import lsbdg
    a = torch.ones(11, dtype=torch.float64, device="cuda:0")
    with pytest.raises(lsbdg.DgError):
        lsbdg.triad(a[:9], a[:9], a[:9], 1.0)
    with pytest.raises(lsbdg.DgError):
        lsbdg.triad(a[1:9], a[2:10], a[2:10], 1.0)
