"""Host checks of the rocprofv3 summary script: which bench stage each kernel
name belongs to (the stage sums and the measured-traffic record depend on it)."""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import rocprof_summary as rs  # noqa: E402

NS = "shtx::(anonymous namespace)::"


def test_classify_gemm_instantiations():
    args = f"({NS}GemmArgs)"
    assert rs.classify(f"void {NS}k_leg_mfma<float, 128, 128, 16, true, 8>{args}") == "legendre_inverse_gemm"
    assert rs.classify(f"void {NS}k_leg_mfma<float, 128, 64, 16, true, 8>{args}") == "legendre_inverse_gemm"
    assert rs.classify(f"void {NS}k_leg_mfma<float, 128, 128, 16, false, 8>{args}") == "legendre_direct_gemm"
    assert rs.classify(f"void {NS}k_leg_mfma<double, 64, 32, 16, false, 4>{args}") == "legendre_direct_gemm"
    assert rs.classify(f"void {NS}k_leg_split<false, 64, 128, 32, true>{args}") == "legendre_inverse_gemm"
    assert rs.classify(f"void {NS}k_leg_split<true, 128, 128, 32, false>{args}") == "legendre_direct_gemm"
    # the split-half form's spectral maximum and the wind step run in the inverse-shaped GEMM stage
    assert rs.classify(f"void {NS}k_uv_spec<float>({NS}Cx<float> const*)") == "legendre_inverse_gemm"
    assert rs.classify(f"void {NS}k_spec_absmax(float2 const*, long, int, unsigned int*)") == "legendre_inverse_gemm"


def test_classify_fft_and_other_kernels():
    args = f"({NS}FftArgs)"
    assert rs.classify(f"void {NS}k_fft_c2r<float, 8192>{args}") == "ring_fft_c2r"
    assert rs.classify(f"void {NS}k_fft_r2c<double, 8192>{args}") == "ring_fft_r2c"
    assert rs.classify("void at::native::vectorized_elementwise_kernel<4, at::native::FillFunctor<float>>") == "copy"
    assert rs.classify(f"void {NS}k_legendre_table<2>(int, double const*)") is None
    assert rs.classify(f"void {NS}k_gauss_nodes(int, double*, double*)") is None
