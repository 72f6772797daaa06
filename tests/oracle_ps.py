"""The oracle's own choice of the lowest order P_S at the library's window, asserted equal to
the library's choice before the oracle's plan is used for a parity comparison (Sec. III-A:
P_S minimises the fitted wavelet's error; Sec. V-A, Fig. MSE2)."""
from functools import lru_cache

from oracle import morlet_oracle as O


@lru_cache(maxsize=None)
def _select(sigma: float, xi: float, K: int, L: int) -> int:
    return O.select_PS(sigma, xi, K, L)


def checked_ps(sigma: float, xi: float, K: int, info: dict) -> int:
    """P_S chosen by the oracle at the window info["L"] the library used; fails unless the
    library chose the same order (info["P_S"])."""
    ps = _select(float(sigma), float(xi), int(K), int(info["L"]))
    assert ps == info["P_S"], ("lowest order differs", sigma, xi, K, info["L"], ps, info["P_S"])
    return ps
