"""Input generator: sizes of the five workloads and consistency of the connectivity with the oracle."""
import numpy as np
import pytest

from meshgen import make_config
from meshgen.columns import column_mesh, random_refined_columns
from oracle import ReferenceElement, build_restriction


def test_config1_sizes():
    m = make_config(1).mesh
    assert (m.n_el, m.n_nodes, m.n_dof) == (128, 1445, 4847)


def test_config2_sizes():
    m = make_config(2).mesh
    assert m.n_el == 78632 and m.n_dof == 6575240
    assert m.refined.sum() == 819


@pytest.mark.parametrize("k", [2, 3, 4])
def test_elem_nodes_agree_with_point_location(k):
    """Conforming slots of elem_nodes are the oracle's unit rows; every hanging slot's row
    only involves nodes of the coarse neighbour face/edge that elem_nodes names for that slot's line."""
    rng = np.random.default_rng(k)
    m = column_mesh(k, 4, 3, 2, refined=random_refined_columns(4, 3, 0.4, rng), extent=(8.0, 6.0, 1.0))
    R = build_restriction(m, ReferenceElement(k)).tocsr()
    S = (k + 1) ** 3
    hang = (m.cmask >> 3) != 0
    for e in range(m.n_el):
        for s in range(S):
            row = R.getrow(e * S + s)
            cols = row.indices[np.abs(row.data) > 1e-14]
            if not hang[e]:
                assert cols.tolist() == [m.elem_nodes[e, s]]
    # hanging elements: the set of nodes touched by R_e equals the set named in elem_nodes
    for e in np.nonzero(hang)[0]:
        Re = R[e * S:(e + 1) * S]
        touched = set(Re.indices[np.abs(Re.data) > 1e-14].tolist())
        assert touched == set(m.elem_nodes[e].tolist())


def test_dmask_base_only():
    w = make_config(2, nx=4, ny=4, nz=2)
    m = w.mesh
    assert m.dmask[2].sum() > 0 and m.dmask[:2].sum() == 0
    assert np.all(m.node_logical[m.dmask[2] == 1, 2] == 0.0)
