"""The Python binding refuses arrays of unequal lengths (and an adjoint length that is not
the line set's) before any library call: a short array would otherwise make the library
read or write past its end.  Runs without a GPU: the device-tensor check is bypassed and
the library handle is a recorder that fails the test if it is called."""
import pytest
import torch

from paper_1801_09803_amd import binding


class _NoCalls:
    def __getattr__(self, name):
        raise AssertionError(f"library call {name} reached despite invalid arguments")


def _plan():
    p = binding.Plan.__new__(binding.Plan)
    p._torch = torch
    p._lib = _NoCalls()
    p._h = None
    p._pid = -1
    p.n_points = 11
    p.dtype = torch.float32
    p.precision = "fp32"
    p._dev = lambda t, dtype, name: t
    p._stream = lambda: None
    return p


def _i(n):
    return torch.zeros(n, dtype=torch.int32)


def _f(n):
    return torch.zeros(n, dtype=torch.float32)


@pytest.mark.parametrize("lens", [(10, 9, 10, 10, 10), (10, 10, 9, 10, 10), (10, 10, 10, 11, 10),
                                  (10, 10, 10, 10, 3)])
def test_set_lines_rejects_unequal_lengths(lens):
    p = _plan()
    u, l, a, g, n = lens
    with pytest.raises(ValueError):
        p.set_lines(_i(u), _i(l), _f(a), _f(g), _f(n))


def test_set_states_rejects_unequal_lengths():
    p = _plan()
    with pytest.raises(ValueError):
        p.set_states(torch.zeros(5, dtype=torch.float64), _i(4), _i(5))
    with pytest.raises(ValueError):
        p.set_states(torch.zeros(5, dtype=torch.float64), _i(5), _i(6))


def test_state_reductions_reject_unequal_lengths():
    p = _plan()
    p._states = (torch.zeros(5, dtype=torch.float64), _i(5), _i(5))
    with pytest.raises(ValueError):
        p.lifetimes(_i(7), _f(6))
    with pytest.raises(ValueError):
        p.cooling_function(_i(7), _i(6), _f(7), [300.0])
    with pytest.raises(ValueError):
        p.cooling_function(_i(7), _i(7), _f(8), [300.0])
    with pytest.raises(ValueError):
        p.set_vibrational_labels(_i(4), 2)


def test_adjoint_needs_the_line_set_length():
    p = _plan()
    g = _f(11)
    with pytest.raises(ValueError):          # no line set yet
        p.cross_section_adjoint(300.0, 1.0, g)
    p._n_lines = 10
    with pytest.raises(ValueError):          # a different count than the line set's
        p.cross_section_adjoint(300.0, 1.0, g, 9)
    with pytest.raises(ValueError):          # grad_sigma must cover the grid
        p.cross_section_adjoint(300.0, 1.0, _f(10), 10)


def test_stream_chunk_rejects_unequal_lengths():
    p = _plan()
    st = binding.Stream.__new__(binding.Stream)
    st._plan, st._lib, st._h, st._pid, st._held = p, _NoCalls(), None, -1, []
    with pytest.raises(ValueError):
        st.chunk(_i(8), _i(8), _f(7))
    with pytest.raises(ValueError):
        st.chunk(_i(8), _i(8), _f(8), _f(8), _f(9))
