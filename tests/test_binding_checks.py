"""CPU checks of the Python binding: a matrix that does not fit the handle (shape, layout,
dtype, device) is rejected before any library call could launch a kernel on it."""
from types import SimpleNamespace

import pytest
import torch

import paper_2405_05865_amd as msp


def _psd(n=64):
    return SimpleNamespace(structure="psd", m=n, n=n, s=8, lam=0.1, handle=None)


def _general(m=80, n=64):
    return SimpleNamespace(structure="general", m=m, n=n, s=8, lam=0.0, handle=None)


def _vec(n, k=None):
    return torch.zeros((n,) if k is None else (k, n), dtype=torch.float64)


@pytest.mark.parametrize("shape", [(63, 64), (64, 65), (64,), (64, 64, 1)])
def test_solve_rejects_wrong_shape(shape):
    A = torch.zeros(shape, dtype=torch.float64)
    with pytest.raises(ValueError, match="shape|2-D"):
        msp.solve(_psd(), A, _vec(64))


def test_solve_rejects_column_major_and_short_ld():
    A = torch.zeros((64, 64), dtype=torch.float64).t()
    A = A[:, :64]
    with pytest.raises(ValueError, match="row-major|leading"):
        msp.solve(_psd(), torch.zeros((64, 128), dtype=torch.float64)[:, ::2], _vec(64))


def test_solve_rejects_host_matrix():
    with pytest.raises(ValueError, match="CUDA"):
        msp.solve(_psd(), torch.zeros((64, 64), dtype=torch.float64), _vec(64))


def test_solve_rejects_bad_dtype_and_bf16_high_matrix():
    with pytest.raises(TypeError):
        msp.solve(_psd(), torch.zeros((64, 64), dtype=torch.float16), _vec(64))
    with pytest.raises(TypeError, match="A_hi"):
        msp.solve(_psd(), torch.zeros((64, 64), dtype=torch.bfloat16), _vec(64))


def test_solve_rejects_mismatched_low_matrix():
    A = torch.zeros((64, 64), dtype=torch.float64)
    with pytest.raises(ValueError, match="shape"):
        msp.solve(_psd(), A, _vec(64), A_lo=torch.zeros((64, 32), dtype=torch.float32))


def test_general_handle_needs_m_by_n():
    with pytest.raises(ValueError, match=r"\(80, 64\)"):
        msp.solve(_general(), torch.zeros((64, 64), dtype=torch.float64), _vec(80))


def test_backward_and_schatten_check_the_matrix():
    with pytest.raises(ValueError, match="shape"):
        msp.solve_backward(_psd(), torch.zeros((32, 32), dtype=torch.float64), _vec(64), _vec(64))
    with pytest.raises(ValueError, match="shape|row-major"):
        msp.schatten(_general(64, 64), torch.zeros((64, 128), dtype=torch.float64)[:, ::2], _vec(64, 4))


def test_batched_checks_every_system():
    good = torch.zeros((64, 64), dtype=torch.float64)
    bad = torch.zeros((64, 63), dtype=torch.float64)
    with pytest.raises(ValueError, match="shape"):
        msp.solve_batched([(_psd(), bad, None, _vec(64, 2)), (_psd(), good, None, _vec(64, 2))])
    with pytest.raises(ValueError, match="shape"):
        msp.solve_batched_backward([(_psd(), bad, None)], [_vec(64, 2)], [_vec(64, 2)])


@pytest.mark.parametrize("autotune", [False, True])
def test_sketch_checks_the_matrix(autotune):
    # a host matrix or a column-major view never reaches msp_sketch / msp_sketch_autotune
    with pytest.raises(ValueError, match="CUDA|HIP"):
        msp.sketch(torch.zeros((64, 64), dtype=torch.float64), 8, 4, 1, autotune=autotune)
    with pytest.raises(ValueError, match="row-major"):
        msp.sketch(torch.zeros((64, 64), dtype=torch.float64).t(), 8, 4, 1, autotune=autotune)
