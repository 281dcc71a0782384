"""Host-side logic of bench.py (no GPU): the peak each kernel class is measured against and
the description of what the matrix cores compute must agree for every precision and
product mode, since the JSON line reports both."""
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_split_peak_is_a_sixth_of_bf16(bench):
    bf16 = bench.PEAK["bf16"]
    for kind in ("conv", "mix_deep"):
        peak, basis = bench.mfma_peak(kind, "fp32", "split3", 64)
        assert peak == pytest.approx(bf16 / 6) and "/ 6" in basis
    # narrow models mix channels on the float matrix cores even in the split mode
    assert bench.mfma_peak("mix_deep", "fp32", "split3", 16)[0] == bench.PEAK["fp32"]
    assert bench.mfma_peak("conv", "fp32", "fp32", 64)[0] == bench.PEAK["fp32"]
    assert bench.mfma_peak("conv", "fp64", "split3", 64)[0] == bench.PEAK["fp64"]
    # BF16-mixed models: hi + lo splits, three bf16 products per product
    assert bench.mfma_peak("mix_deep", "bf16", "split3", 64)[0] == pytest.approx(bf16 / 3)
    assert bench.mfma_peak("conv", "bf16", "split3", 64)[0] == pytest.approx(bf16 / 3)


@pytest.mark.parametrize("prec,products,d", [(p, m, d) for p in ("fp32", "bf16", "fp64")
                                              for m in ("split3", "fp32") for d in (16, 64)])
def test_products_label_matches_peaks(bench, prec, products, d):
    label = bench.products_label(prec, products, d)
    if prec == "fp64":
        assert label == "f64 matrix cores"
        return
    toeplitz, mix = label.split("; channel mixing: ")
    conv_basis = bench.mfma_peak("conv", prec, products, d)[1]
    assert ("three-term" in toeplitz) == ("/ 6" in conv_basis)
    assert ("hi + lo" in toeplitz) == ("/ 3" in conv_basis)
    deep_peak, deep_basis = bench.mfma_peak("mix_deep", prec, products, d)
    if prec == "bf16" and d > 16:
        assert mix.startswith("hi + lo") and deep_peak == pytest.approx(bench.PEAK["bf16"] / 3)
    elif products == "split3" and d > 16:
        assert "three-term" in mix and "/ 6" in deep_basis
    else:
        assert mix == "f32 matrix cores" and deep_peak == bench.PEAK["fp32"]


@pytest.mark.parametrize("name,cls", [
    ("void dn::deep_kernel<float, 64, true, false, 3, 16>(dn::MixArgs<float>)", "mix_deep"),
    ("void dn::inject_add_kernel<float, 64>(dn::MixArgs<float>)", "mix_deep"),
    ("void dn::inject_w1_kernel<float, 64>(dn::MixArgs<float>)", "conv"),
    ("void dn::conv_split_kernel<4, 3>(dn::ConvArgs<float>)", "conv"),
    ("void dn::last_finish_kernel<float, 64, true>(dn::MixArgs<float>)", "tail"),
    ("void dn::slice_mma_kernel<float, 64, true>(dn::SliceArgs<float>)", "slice"),
    ("void dn::mix_kernel<float, 64, 1, false>(dn::MixArgs<float>)", "mix_tau"),
    ("dn::sr_rowdot_part_kernel<float>(float const*, long, int, double const*, double*)", "other"),
])
def test_kernel_class_of_profiler_names(bench, name, cls):
    # the grouping the profile summaries and the roofline use, including the kernels of the
    # phi-injected path (block 1's mixer output counts with the Toeplitz products it replaces)
    assert bench.kernel_class(name) == cls
