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


def _counter_db(path, rows):
    """A --pmc results database with the columns profile_summary reads."""
    import sqlite3
    c = sqlite3.connect(path)
    c.execute("create table counters_collection (kernel_name text, dispatch_id int, counter_name text, "
              "value real, grid_size_x int, workgroup_size_x int, grid_size_y int, grid_size_z int)")
    c.executemany("insert into counters_collection values (?,?,?,?,?,?,?,?)", rows)
    c.commit()
    c.close()


def test_counter_table_scales_by_the_copy_kernel(tmp_path):
    """FETCH_SIZE (KiB per dispatch) becomes bytes through the copy kernel's
    reading in the same run (its first dispatch only writes and is skipped);
    counters are averaged per kernel and grid, and a counter summed over
    several rows of one dispatch (per-XCD instances) counts once per dispatch."""
    from paper_2003_11069_amd.profile_summary import counters_table
    copy = 1 << 20  # bytes read and written per copy dispatch
    rows = [("k_copy_probe", 0, "FETCH_SIZE", 5.0, 256, 256, 1, 1)]
    rows += [("k_copy_probe", d, "FETCH_SIZE", copy / 1024 / 2, 256, 256, 1, 1) for d in (1, 2, 3)]
    # k_x on two grids; dispatch 10 reports FETCH_SIZE in two halves
    rows += [("void k_x<1>(A)", 10, "FETCH_SIZE", 30.0, 512, 256, 1, 1),
             ("void k_x<1>(A)", 10, "FETCH_SIZE", 10.0, 512, 256, 1, 1),
             ("void k_x<1>(A)", 11, "FETCH_SIZE", 60.0, 512, 256, 1, 1),
             ("void k_x<1>(A)", 12, "FETCH_SIZE", 8.0, 1024, 256, 2, 1),
             ("void k_x<1>(A)", 12, "SQ_WAVES", 64.0, 1024, 256, 2, 1)]
    db = tmp_path / "p.db"
    _counter_db(str(db), rows)
    out, scale = counters_table([str(db)], "k_x", copy)
    assert scale["FETCH_SIZE"] == 2.0
    got = {g: (n, m) for _, g, n, m in out}
    assert got[(2, 1, 1)] == (2, {"FETCH_SIZE": (40.0 + 60.0) / 2 * 1024 * 2.0})
    assert got[(4, 2, 1)] == (1, {"FETCH_SIZE": 8.0 * 1024 * 2.0, "SQ_WAVES": 64.0})
