"""Host-side checks of the Python binding (no GPU): wrong output or workspace
tensors are refused before any pointer reaches the library."""

import pytest

torch = pytest.importorskip("torch")

from paper_1712_07070_amd import hydro  # noqa: E402


def lvl(G, dtype=torch.float64):
    return torch.zeros((G, 5, 16, 16, 16), dtype=dtype)


@pytest.mark.parametrize("bad_out", [
    lambda: lvl(1, torch.float32),                       # dtype differs from the state
    lambda: lvl(2),                                      # one group too many
    lambda: torch.zeros((1, 5, 16, 16, 15), dtype=torch.float64),
])
def test_level_adjoint_rejects_wrong_out(bad_out):
    with pytest.raises(ValueError):
        hydro.advance_level_adjoint(lvl(1), lvl(1), (1, 1, 1), (0,) * 6, 1e-3, 0.1, 1.4, out=bad_out())
    with pytest.raises(ValueError):
        hydro.autotune_adjoint(lvl(1), lvl(1), (1, 1, 1), (0,) * 6, 0.1, 1.4, out=bad_out())


def test_padded_adjoint_rejects_wrong_out():
    U = torch.zeros((1, 5, 22, 22, 22), dtype=torch.float64)
    with pytest.raises(ValueError):
        hydro.advance_adjoint(U, lvl(1), 1e-3, 0.1, 1.4, out=torch.zeros((1, 5, 20, 20, 20), dtype=torch.float64))
    with pytest.raises(ValueError):
        hydro.advance_adjoint(U, lvl(1), 1e-3, 0.1, 1.4, out=U.float())


def test_adjoint_rejects_non_byte_workspace():
    with pytest.raises(ValueError):
        hydro.advance_level_adjoint(lvl(1), lvl(1), (1, 1, 1), (0,) * 6, 1e-3, 0.1, 1.4,
                                    work=torch.zeros(16, dtype=torch.float64))
