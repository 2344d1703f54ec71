"""The library's marching-cubes case table (built on the host by its own
implementation of the face-walk construction) equals the oracle's."""
from oracle import tsdf as ot
from paper_2509_17390_amd import rcast


def test_library_case_table_equals_the_oracle_table():
    count, tris = rcast.marching_cubes_table()
    tab = ot.table()
    for c in range(256):
        assert count[c] == len(tab[c]), c
        got = [tuple(int(x) for x in tris[c, 3 * k:3 * k + 3]) for k in range(count[c])]
        assert got == [tuple(t) for t in tab[c]], c
        assert all(tris[c, 3 * count[c]:] == -1)
