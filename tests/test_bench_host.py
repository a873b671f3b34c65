"""Host-side checks of bench.py's byte accounting (no GPU).  The algorithmic
bytes per fluid-node update are rebuilt here from the lattice size and the
element widths: the paper's two-population state (each component's
populations read and written once, psi written and read once: 152 / 80 B for
D2Q9 in 4- / 2-byte storage, 440 / 224 B for D3Q27) and the library's k_main
(deviations read and written, rho1 and psi read, the colour fraction a and
the colour vector B written)."""
import bench


def test_two_population_state_bytes():
    for dim, q in ((2, 9), (3, 27)):
        for storage, e in (("fp32", 4), ("fp32_f32", 4), ("fp16", 2), ("bf16", 2)):
            assert bench.two_pop_bytes(dim, storage) == 2 * 2 * q * e + 2 * 4
    assert (bench.two_pop_bytes(2, "fp32"), bench.two_pop_bytes(2, "bf16")) == (152, 80)
    assert (bench.two_pop_bytes(3, "fp32"), bench.two_pop_bytes(3, "fp16")) == (440, 224)


def test_main_kernel_bytes():
    # FP32 storage: 27 FP32 deviations each way, rho1 and psi read in FP64,
    # a written in FP64, B written as 3 FP32
    assert bench.main_kernel_bytes(3, "fp32") == 2 * 27 * 4 + 2 * 8 + 8 + 3 * 4 == 252
    # 16-bit storage: 26 deviations at 2 B plus the FP32 rest slot each way,
    # FP32 rho1, psi and a, B as 3 FP32
    for storage in ("fp16", "bf16"):
        assert bench.main_kernel_bytes(3, storage) == 2 * (26 * 2 + 4) + 2 * 4 + 4 + 3 * 4 == 136
    # D2Q9 FP32: 9 deviations each way, FP64 rho1, psi, a, B as 2 FP32
    assert bench.main_kernel_bytes(2, "fp32") == 2 * 9 * 4 + 2 * 8 + 8 + 2 * 4
