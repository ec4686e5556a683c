"""Host logic of the world partitioning used to run a batch on several streams."""
import pytest

from paper_2310_07854_amd.optim import split_worlds


@pytest.mark.parametrize("n,p", [(64, 4), (4, 3), (5, 2), (3, 8), (1, 1), (7, 7)])
def test_split_worlds_covers_every_world_once(n, p):
    r = split_worlds(n, p)
    assert len(r) == min(n, p)
    assert r[0][0] == 0 and r[-1][1] == n
    assert all(a[1] == b[0] for a, b in zip(r, r[1:]))
    sizes = [b - a for a, b in r]
    assert min(sizes) >= 1 and max(sizes) - min(sizes) <= 1


def test_split_worlds_rejects_empty():
    with pytest.raises(ValueError):
        split_worlds(0, 2)
    with pytest.raises(ValueError):
        split_worlds(3, 0)
