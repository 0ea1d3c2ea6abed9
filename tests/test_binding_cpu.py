"""Argument checks of the Python binding, on the host: tensors that would
make a kernel read or write past an allocation are refused before any call
crosses the C ABI."""
import pytest
import torch

from paper_1801_04348_amd import pk
from tests import machines


@pytest.fixture(scope="module")
def table():
    return pk.pk_case_table_build(0, machines.gfx950())


def test_expanded_operand_is_refused(table):
    A = torch.zeros(1, 8).expand(16, 8)          # row stride 0: every row aliases the first
    B = torch.zeros(8, 4)
    C = torch.zeros(16, 4)
    with pytest.raises(ValueError, match="rows overlap"):
        pk.pk_matmul(table, None, "f32", A, B, C)


def test_overlapping_output_rows_are_refused(table):
    A = torch.zeros(4, 8)
    B = torch.zeros(8, 6)
    C = torch.zeros(40).as_strided((4, 6), (3, 1))   # rows 3 elements apart, 6 wide
    with pytest.raises(ValueError, match="rows overlap"):
        pk.pk_matmul(table, None, "f32", A, B, C)


def test_element_size_must_match_dtype(table):
    A = torch.zeros(4, 8, dtype=torch.int16)
    B = torch.zeros(8, 6, dtype=torch.int16)
    C = torch.zeros(4, 6)
    with pytest.raises(ValueError, match="2-byte elements"):
        pk.pk_matmul(table, None, "f32", A, B, C)
    with pytest.raises(ValueError, match="4-byte elements"):
        pk.pk_matmul(table, None, "bf16", torch.zeros(4, 8), torch.zeros(8, 6), C)
    with pytest.raises(ValueError, match="C has 2-byte"):
        pk.pk_matmul(table, None, "bf16", A, B, torch.zeros(4, 6, dtype=torch.int16))


def test_host_tensors_are_refused(table):
    A, B, C = torch.zeros(4, 8), torch.zeros(8, 6), torch.zeros(4, 6)
    with pytest.raises(ValueError, match="GPU tensor"):
        pk.pk_matmul(table, None, "f32", A, B, C)
    with pytest.raises(ValueError, match="GPU tensor"):
        pk.pk_madd(table, None, "f32", C, C, C)
    with pytest.raises(ValueError, match="GPU tensor"):
        pk.pk_transpose(table, None, "f32", A, torch.zeros(8, 4))
    with pytest.raises(ValueError, match="GPU tensor"):
        pk.pk_grouped_plan_create(table, "f32", [A], [B], [C])


def test_non_unit_column_stride_is_refused(table):
    A = torch.zeros(8, 4).t()                    # (4, 8) with column stride 4
    with pytest.raises(ValueError, match="unit column stride"):
        pk.pk_matmul(table, None, "f32", A, torch.zeros(8, 6), torch.zeros(4, 6))


def test_learned_margin_bounds(table):
    pk.pk_case_table_set_learned_margin(table, 0.0)
    pk.pk_case_table_set_learned_margin(table, 0.05)
    with pytest.raises(pk.PkError) as e:
        pk.pk_case_table_set_learned_margin(table, -0.1)
    assert e.value.code == pk.PK_ERR_INVALID_ARG
    assert pk.pk_case_table_learned_measured(table) == 0
