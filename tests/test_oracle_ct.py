"""Pins of the oracle's 12-bit CT path (uint16 maps, tables of up to 4096
rows; Section 2.2.2) against its 8-bit path (no GPU): a map read as uint16
gives the same solve as the same map read as uint8, and moving the materials
to high rows of a 4096-row table changes nothing."""
import numpy as np
import pytest

import oracle
import synth


def test_uint16_map_equals_uint8_map():
    case = synth.random_small_case(8, n_steps=40)
    src = oracle.source_plane(case)
    p8 = oracle.problem_from_case(case)
    a, ia, _ = oracle.solve(p8, case.mat, src)
    p16 = oracle.problem_from_case(case, index_bits=16)
    b, ib, _ = oracle.solve(p16, case.mat.astype(np.uint16), src)
    assert np.array_equal(a, b) and ia == ib


def test_materials_at_high_rows_of_a_4096_row_table():
    case = synth.random_small_case(9, n_steps=40)
    src = oracle.source_plane(case)
    a, ia, _ = oracle.solve(oracle.problem_from_case(case), case.mat, src)
    rows = np.array([0, 1000, 2500, 4095])
    table = np.tile(case.materials[0], (4096, 1))
    table[rows] = case.materials
    mat16 = rows[case.mat].astype(np.uint16)
    prob = oracle.problem_from_case(case, index_bits=16, materials=table)
    b, ib, _ = oracle.solve(prob, mat16, src)
    assert np.array_equal(a, b) and ia == ib


def test_4096_rows_need_16_bit_maps():
    case = synth.random_small_case(10, n_steps=5)
    table = np.tile(case.materials[0], (300, 1))
    with pytest.raises(oracle.OracleError):
        oracle.setup(oracle.problem_from_case(case, materials=table))
    oracle.setup(oracle.problem_from_case(case, materials=table, index_bits=16))
    over = np.tile(case.materials[0], (4097, 1))
    with pytest.raises(oracle.OracleError):
        oracle.setup(oracle.problem_from_case(case, materials=over, index_bits=16))
