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
    # factorisation and apply carry the stored factor values (20 per cell)
    assert b.solve_bytes_per_cell(True, 4.0, one(0)) - base == 40 + 20 * 4
    assert b.solve_bytes_per_cell(True, 8.0, one(0)) - base == 40 + 20 * 8
    assert b.solve_bytes_per_cell(True, 4.0, one(1)) - base == 32 + 20 * 4
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
