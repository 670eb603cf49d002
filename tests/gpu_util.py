"""Helpers shared by the GPU tests: run the HIP path through the binding and
compare with the oracle element by element."""
import numpy as np
import torch

import oracle


def to_dev(g):
    return torch.from_numpy(np.ascontiguousarray(g.edges, dtype=np.int32)).cuda()


def gpu_all(bfc, g, tuning=None):
    """(total, wedges, per-vertex upper, per-vertex lower, per-edge) from the HIP library."""
    with bfc.Graph(to_dev(g), g.n_upper, g.n_lower) as h:
        if tuning:
            h.set_tuning(**tuning)
        tot, wed = h.count_total()
        up, lo = h.count_per_vertex()
        be = h.count_per_edge()
        torch.cuda.synchronize()
        return tot, wed, up.cpu().numpy(), lo.cpu().numpy(), be.cpu().numpy()


def check_against_oracle(bfc, g, tuning=None, wedges=True):
    tot, wed, up, lo, be = gpu_all(bfc, g, tuning)
    o_tot = oracle.total(g)
    o_up, o_lo = oracle.vertex_counts(g)
    o_be = oracle.edge_counts(g)
    assert tot == o_tot, (g.name, tot, o_tot)
    np.testing.assert_array_equal(up, o_up)
    np.testing.assert_array_equal(lo, o_lo)
    np.testing.assert_array_equal(be, o_be)
    if wedges:
        assert wed == oracle.vp_wedges(g), g.name
    return tot
