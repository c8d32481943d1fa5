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


def _problem(spv, n, row_ptr, col, J, h, colour, n_colours, nnz=None):
    import torch
    t = lambda a, dt: torch.as_tensor(np.asarray(a, dtype=dt)).cuda()
    rp = np.asarray(row_ptr, np.int32)
    return spv.Problem(n, int(rp[-1]) if nnz is None else nnz, t(rp, np.int32), t(col if len(col) else [0], np.int32),
                       t(J if len(J) else [0], np.int32), t(h, np.int32), t(colour, np.uint8), n_colours, 0)


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


def test_bounds_are_derived_by_the_library(spv, ctx):
    """The ABI takes no degree or field bound from the caller: the library derives both at
    ingest (the longest row and max_i |h_i| + sum_j |J_ij|) and returns them."""
    import ctypes
    names = [f[0] for f in spv.spv_problem._fields_]
    assert "x_bound" not in names and "max_degree" not in names
    assert ctypes.sizeof(spv.spv_problem) == 4 * 2 + 8 * 5 + 4 * 2
    assert spv.spv_problem_check(ctx, _problem(spv, **OK)) == (2, 5)  # row 1: |h_1| + 2 + 3 = 5
    inst = si.cubic_lattice(4, "gauss", seed=5, scale_log2=10)
    rows = np.repeat(np.arange(inst.n), np.diff(inst.row_ptr))
    x = np.abs(inst.h).astype(np.int64)
    np.add.at(x, rows, np.abs(inst.J))
    assert spv.spv_problem_check(ctx, spv.Problem.from_instance(inst)) == (6, int(x.max()))


def test_field_bound_at_2_26_rejected(spv, ctx):
    # |h_0| + |J_01| = 2^26 exceeds the three base-512 digits of the acceptance test
    P = _problem(spv, 2, [0, 1, 2], [1, 0], [1, 1], [2**26 - 1, 0], [0, 1], 2)
    assert _code(spv, ctx, P) == ERANGE
    P = _problem(spv, 2, [0, 1, 2], [1, 0], [1, 1], [2**26 - 2, 0], [0, 1], 2)
    assert spv.spv_problem_check(ctx, P) == (1, 2**26 - 1)


def test_sampling_calls_ingest(spv, ctx):
    """A sampling call refuses a malformed instance before launching (the same ingest), and
    samples a valid one with the bounds it derived: two-digit tables on the Gaussian cube,
    bit-identical to the oracle."""
    import oracle
    bad = _problem(spv, **_with(colour=[0, 0, 1]))
    with pytest.raises(spv.SpvError) as e:
        spv.spv_sample(ctx, bad, si.linear_betas(0.1, 1.0, 5), 4, 1)
    assert e.value.code == ECOLOUR
    inst = si.cubic_lattice(4, "gauss", seed=6, scale_log2=10)
    betas = si.linear_betas(0.2, 3.0, 40)
    sp, E = spv.spv_sample(ctx, spv.Problem.from_instance(inst), betas, 9, 77)
    osp, oE = oracle.sa_sample(inst, betas, reads=9, seed=77)
    assert np.array_equal(sp.cpu().numpy(), osp) and np.array_equal(E.cpu().numpy(), oE)


def test_row_beyond_64_entries_rejected(spv, ctx):
    n = 66  # a star: variable 0 joined to 65 leaves
    rp = np.r_[0, 65, 66 + np.arange(65)]
    col = np.r_[np.arange(1, 66), np.zeros(65, int)]
    P = _problem(spv, n, rp, col, np.ones(130), np.zeros(n), np.r_[0, np.ones(65)], 2)
    assert _code(spv, ctx, P) == ECAPACITY


def test_too_many_variables_rejected(spv, ctx):
    import torch
    z = torch.zeros(1, dtype=torch.int32).cuda()
    P = spv.Problem(70000, 0, z, z, z, z, torch.zeros(1, dtype=torch.uint8).cuda(), 1, 0)
    assert _code(spv, ctx, P) == ECAPACITY
