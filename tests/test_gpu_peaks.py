"""The library's peak microbenchmarks (oz_peak): every kind returns a rate in
the range the MI355X's vendor figures allow (and well above a fraction of
them, so a kernel that did no work would fail), and bad arguments are refused
before anything runs."""
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def oz():
    import paper_2503_22875_amd as mod
    return mod


@pytest.fixture(scope="module")
def handle(oz):
    torch.cuda.set_device(0)
    h = oz.oz_create(0)
    oz.oz_set_stream(h, torch.cuda.current_stream().cuda_stream)
    yield h
    oz.oz_destroy(h)


def test_peak_rates_are_plausible(oz, handle):
    print("oz_peak kinds 0..4", flush=True)
    i8 = oz.oz_peak(handle, 0, 2000)
    i8_16 = oz.oz_peak(handle, 3, 2000)
    i8_rand = oz.oz_peak(handle, 4, 2000)
    f64 = oz.oz_peak(handle, 1, 2000)
    src = torch.ones(1 << 24, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    cp = oz.oz_peak(handle, 2, 4, src, dst, src.numel() * 8)
    torch.cuda.synchronize()
    print("int8 %.0f / %.0f / %.0f TOP/s, fp64 %.1f TFLOP/s, copy %.0f GB/s"
          % (i8 / 1e12, i8_16 / 1e12, i8_rand / 1e12, f64 / 1e12, cp / 1e9))
    assert 1.0e15 < i8 <= 5.0e15 * 1.05       # vendor dense INT8: 5.0 POP/s
    assert 1.0e15 < i8_16 <= 5.0e15 * 1.05
    assert 1.0e15 < i8_rand <= 5.0e15 * 1.05
    assert 1.0e13 < f64 <= 78.6e12 * 1.05     # vendor FP64 matrix: 78.6 TFLOP/s
    assert 1.0e12 < cp <= 8.0e12 * 1.05       # vendor HBM: 8 TB/s
    # the copy really copied
    assert torch.equal(dst, src)


def test_peak_argument_errors(oz, handle):
    src = torch.ones(64, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for args in [(5, 10, None, None, 0), (-1, 10, None, None, 0), (0, 0, None, None, 0),
                 (2, 1, src, dst, 0), (2, 1, src, dst, 24), (2, 1, None, dst, 512)]:
        with pytest.raises(oz.OzError):
            oz.oz_peak(handle, *args)
