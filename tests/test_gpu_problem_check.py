"""The boundary's validation of a problem (spv_problem_check, synchronous): every malformed
CSR, colouring or range is rejected with its status code, a valid problem passes."""
import numpy as np
import pytest

import spvar_inputs as si

pytestmark = pytest.mark.gpu

EINVAL, EASYM, ECOLOUR, ERANGE, ECAPACITY = -1, -2, -3, -4, -5


@pytest.fixture(scope="module")
def spv():
    import paper_1706_07826_amd as m
    return m


@pytest.fixture(scope="module")
def ctx(spv):
    return spv.Context(0)


def _problem(spv, n, row_ptr, col, J, h, colour, n_colours, max_degree=None, x_bound=None, nnz=None):
    import torch
    t = lambda a, dt: torch.as_tensor(np.asarray(a, dtype=dt)).cuda()
    rp = np.asarray(row_ptr, np.int32)
    deg = np.diff(rp)
    md = max_degree if max_degree is not None else max(1, int(deg.max()) if n else 1)
    if x_bound is None:
        rows = np.repeat(np.arange(n), deg)
        s = np.zeros(n, np.int64)
        np.add.at(s, rows, np.abs(np.asarray(J, np.int64)))
        x_bound = int((np.abs(np.asarray(h, np.int64)) + s).max()) if n else 0
    return spv.Problem(n, int(rp[-1]) if nnz is None else nnz, t(rp, np.int32), t(col if len(col) else [0], np.int32),
                       t(J if len(J) else [0], np.int32), t(h, np.int32), t(colour, np.uint8), n_colours, 0, md,
                       x_bound)


def _code(spv, ctx, P):
    with pytest.raises(spv.SpvError) as e:
        spv.spv_problem_check(ctx, P)
    return e.value.code


# a valid 3-path 0-1-2 with couplers 2 and -3, two colours
OK = dict(n=3, row_ptr=[0, 1, 3, 4], col=[1, 0, 2, 1], J=[2, 2, -3, -3], h=[1, 0, -1], colour=[0, 1, 0], n_colours=2)


def _with(**kw):
    d = dict(OK)
    d.update(kw)
    return d


def test_valid_problem_passes(spv, ctx):
    spv.spv_problem_check(ctx, _problem(spv, **OK))
    inst = si.chimera(4, seed=3)
    spv.spv_problem_check(ctx, spv.Problem.from_instance(inst))


@pytest.mark.parametrize("name,kw,code", [
    ("asymmetric_J", dict(J=[2, 3, -3, -3]), EASYM),
    ("missing_transpose", dict(row_ptr=[0, 1, 2, 3], col=[1, 2, 1], J=[2, -3, -3]), EASYM),
    ("self_loop", dict(row_ptr=[0, 1, 3, 4], col=[1, 1, 2, 1], J=[2, 2, -3, -3]), EASYM),
    ("unsorted_row", dict(col=[1, 2, 0, 1], J=[2, -3, 2, -3]), EASYM),
    ("col_out_of_range", dict(col=[1, 0, 3, 1]), EASYM),
    ("row_ptr_end", dict(nnz=3), EASYM),
    ("edge_inside_colour", dict(colour=[0, 0, 1]), ECOLOUR),
    ("colour_past_count", dict(colour=[0, 2, 0]), ECOLOUR),
    ("coupler_range", dict(J=[40000, 40000, -3, -3]), ERANGE),
])
def test_malformed_problem_rejected(spv, ctx, name, kw, code):
    assert _code(spv, ctx, _problem(spv, **_with(**kw))) == code


def test_understated_bounds_rejected(spv, ctx):
    assert _code(spv, ctx, _problem(spv, **OK, x_bound=3)) == ERANGE  # true bound |h_1| + 2 + 3 = 5
    assert _code(spv, ctx, _problem(spv, **OK, max_degree=1)) == EINVAL  # row 1 has two entries


def test_too_many_variables_rejected(spv, ctx):
    import torch
    z = torch.zeros(1, dtype=torch.int32).cuda()
    P = spv.Problem(70000, 0, z, z, z, z, torch.zeros(1, dtype=torch.uint8).cuda(), 1, 0, 1, 0)
    assert _code(spv, ctx, P) == ECAPACITY
