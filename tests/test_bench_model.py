"""Host-side checks of bench.py's algorithmic byte model (no GPU): the bytes
per cell of a column-step follow from the phases it executed."""
import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


def bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(HERE, "..", "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_settled_column_costs_the_set_up_only():
    b = bench()
    assert b.solve_bytes_per_cell(False, 4.0, np.zeros(8, np.int32)) == 72.0
    assert b.solve_bytes_per_cell(True, 4.0, np.zeros(8, np.int32)) == 104.0


def test_phase_bytes():
    b = bench()
    one = lambda i: np.eye(8, dtype=np.int32)[i]
    base = b.solve_bytes_per_cell(True, 4.0, np.zeros(8, np.int32))
    # factorisation and apply carry the stored factor values (16 per cell)
    assert b.solve_bytes_per_cell(True, 4.0, one(0)) - base == 40 + 16 * 4
    assert b.solve_bytes_per_cell(True, 8.0, one(0)) - base == 40 + 16 * 8
    assert b.solve_bytes_per_cell(True, 4.0, one(1)) - base == 32 + 16 * 4
    assert b.solve_bytes_per_cell(True, 4.0, one(2)) - base == 104
    assert b.solve_bytes_per_cell(True, 4.0, one(3)) - base == 120
    # a CGS pass over k basis vectors: w in and out plus 16 B per vector
    k = 5
    c = np.zeros(8, np.int32)
    c[4], c[6] = 1, k
    assert b.solve_bytes_per_cell(True, 4.0, c) - base == 32 + 16 * k
    # a learned candidate's residual
    assert b.solve_bytes_per_cell(True, 4.0, one(7)) - base == 72


def test_gather_and_write_back_bytes():
    b = bench()
    assert b.gather_bytes_per_cell(True) - b.gather_bytes_per_cell(False) == 32
    assert b.WRITEBACK_BYTES_PER_CELL == 32


def test_factor_values_follow_the_device_layout():
    """The model's factor bytes use the number of block-factor values the
    kernels store per cell: the device's factor slots minus the four
    approximate-Schur couplings, read from the kernel headers."""
    import re
    b = bench()
    src = open(os.path.join(HERE, "..", "paper_1904_08510_amd", "csrc", "jfnk_types.h")).read()
    slots = int(re.search(r"constexpr int kFactorSlots = (\d+);", src).group(1))
    base = b.solve_bytes_per_cell(False, 4.0, np.zeros(8, np.int32))
    one = lambda i: np.eye(8, dtype=np.int32)[i]
    for fb in (4.0, 8.0):
        assert b.solve_bytes_per_cell(False, fb, one(0)) - base == 40 + (slots - 4) * fb
        assert b.solve_bytes_per_cell(False, fb, one(1)) - base == 32 + (slots - 4) * fb

