"""CPU checks of the C-ABI library: it loads and exports every declared symbol, its plan matches the
oracle's block partition, its host-built labels match the oracle's f_s L, and the float64 validation hook
(same index arithmetic as the GPU kernel) reproduces the oracle's block updates."""
import os
import re

import numpy as np
import pytest

from oracle import blockbp, lattice, mps, network
from paper_2402_04834_amd import workload

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bbp():
    import paper_2402_04834_amd as pkg
    from paper_2402_04834_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libbbp.so is not built (run `python -m paper_2402_04834_amd.build`)")
    return pkg


def test_library_exports_every_declared_symbol(bbp):
    from paper_2402_04834_amd import _lib
    header = open(os.path.join(ROOT, "include", "bbp.h")).read()
    declared = set(re.findall(r"\b(bbp_[a-z_]+)\s*\(", header))
    declared -= {"bbp_opts", "bbp_net", "bbp_timing", "bbp_plan_info"}
    h = _lib.lib()
    for name in sorted(declared):
        assert hasattr(h, name), name
    assert declared <= set(_lib.SIGNATURES)


@pytest.mark.parametrize("d,k,chi", [(5, 3, 4), (11, 4, 16), (17, 6, 32), (21, 6, 32), (25, 6, 32)])
def test_plan_matches_oracle_partition_and_is_exact(bbp, d, k, chi):
    info = bbp.plan_query(d, bbp.default_opts(block=k, chi=chi))
    p = blockbp.Plan(d, k, k)
    assert info.num_messages == p.M
    assert (info.block_grid_rows, info.block_grid_cols) == (p.nI, p.nJ)
    # every configuration in scope has block boundary states of rank <= chi: the truncation never acts
    assert info.exact_sweeps == 1 and info.gpu_supported == 1


def test_plan_detects_binding_truncation(bbp):
    # chi below the boundary rank of a 6x6 block: those sweeps (and only those) take the truncating kernel
    info = bbp.plan_query(7, bbp.default_opts(block=6, chi=8))
    assert info.exact_sweeps == 0 and info.max_cut_rank == 16 and info.gpu_supported == 1
    assert 0 < info.truncating_sweeps and info.message_stride == 64
    info = bbp.plan_query(7, bbp.default_opts(block=6, chi=16))
    assert info.exact_sweeps == 1 and info.truncating_sweeps == 0


@pytest.mark.parametrize("d,k,chi,stride", [(9, 7, 16, 128), (9, 8, 16, 256), (17, 8, 16, 256)])
def test_wide_blocks_run_every_sweep_in_the_truncating_kernel(bbp, d, k, chi, stride):
    info = bbp.plan_query(d, bbp.default_opts(block=k, chi=chi))
    p = blockbp.Plan(d, k, k)
    assert info.gpu_supported == 1 and info.message_stride == stride
    assert info.truncating_sweeps == p.M + p.nI * p.nJ        # every update and every closing sweep
    assert info.max_cut_rank > chi                              # the truncation really acts


@pytest.mark.parametrize("d,k,chi,why", [(9, 9, 16, "larger than 8"), (9, 8, 32, "up to 16"),
                                         (9, 6, 4, "message MPSs")])
def test_unsupported_truncation_is_refused_with_a_reason(bbp, d, k, chi, why):
    from paper_2402_04834_amd import _lib
    info = bbp.plan_query(d, bbp.default_opts(block=k, chi=chi))
    assert info.gpu_supported == 0
    assert why in _lib.lib().bbp_last_error().decode()


def test_invalid_arguments_are_rejected(bbp):
    from paper_2402_04834_amd import _lib
    with pytest.raises(_lib.BbpError):
        bbp.build_network(3, 0.1, np.zeros(5, dtype=np.uint8))
    with pytest.raises(_lib.BbpError):
        bbp.build_network(3, 1.5, np.zeros(12, dtype=np.uint8))
    with pytest.raises(_lib.BbpError):
        bbp.workspace_size(5, 4, bbp.default_opts(damping=1.5))
    with pytest.raises(_lib.BbpError):
        bbp.workspace_size(5, 4, bbp.default_opts(delta0=1e-1, delta1=1e-3))


@pytest.mark.parametrize("d", [3, 5, 9])
def test_host_network_labels_match_oracle(bbp, d):
    _, s = workload.make_batch(d, 0.1, 5)
    x, z = lattice.coset_labels(d, s)
    for i in range(5):
        lab = bbp.build_network(d, 0.1, s[i]).labels()
        np.testing.assert_array_equal(lab & 1, x[i])
        np.testing.assert_array_equal(lab >> 1, z[i])


def _dense_msgs(plan, rng):
    out = np.zeros((plan.M, 64))
    mps_msgs = {}
    for e, (src, dst, _) in enumerate(plan.edges):
        K = plan.msg_len(src, dst)
        v = rng.uniform(0.05, 1.0, size=2 ** K)
        v /= np.linalg.norm(v)
        v = v.astype(np.float32).astype(np.float64)     # the library stores messages in float32
        out[e, : 2 ** K] = v
        mps_msgs[(src, dst)], _ = mps.canonical_message(mps.from_dense(v[None], [2] * K), 64)
    return out, mps_msgs


@pytest.mark.parametrize("d,k", [(3, 2), (5, 3), (5, 4), (7, 4), (7, 6), (9, 6), (7, 5), (4, 3), (5, 1)])
def test_reference_sweep_matches_oracle(bbp, d, k):
    # every directed update and every closing sweep of the plan, on one coset of one syndrome
    rng = np.random.default_rng(d * 10 + k)
    eps = 0.1
    _, s = workload.make_batch(d, eps, 1)
    x, z = lattice.coset_labels(d, s)
    cos = 2
    labels = (x[0, cos] | (z[0, cos] << 1)).astype(np.uint8)
    L = 2 * d - 1
    # the library holds the noise table in float32 (1 - eps and eps / 3 rounded); use the same numbers
    e32 = np.float32(eps)
    pi32 = np.array([[np.float32(1) - e32, e32 / np.float32(3)], [e32 / np.float32(3)] * 2], dtype=np.float64)
    tensors = network.coset_tensors(d, x[0, cos][None], z[0, cos][None], pi32)
    plan = blockbp.Plan(d, k, k)
    dense, mmsgs = _dense_msgs(plan, rng)
    opts = bbp.default_opts(block=k, chi=64)
    for e, (src, dst, dname) in enumerate(plan.edges):
        got, ls = bbp.reference_update_host(d, eps, opts, labels, e, dense)
        ref, lr = blockbp.block_sweep(plan, tensors, mmsgs, src[0], src[1], dname, 64, (1,))
        refv = mps.to_dense(ref)[0]
        n = refv.size
        np.testing.assert_allclose(got[:n] * np.exp(ls), refv * np.exp(lr[0]), rtol=1e-7,
                                   atol=1e-12 * np.abs(refv).max() * np.exp(lr[0]))
        assert np.all(got[n:] == 0)
    for b, (I, J) in enumerate(plan.blocks):
        got, ls = bbp.reference_update_host(d, eps, opts, labels, -1 - b, dense)
        st, lr = blockbp.block_sweep(plan, tensors, mmsgs, I, J, "E", 64, (1,))
        east = (I, J + 1)
        if plan.has(east):
            w = mps.overlap(st, mmsgs[(east, (I, J))])[0]
            e_id = [q for q, ed in enumerate(plan.edges) if ed[0] == east and ed[1] == (I, J)][0]
            wg = float(np.dot(got[: 2 ** plan.rows[I][1]], dense[e_id, : 2 ** plan.rows[I][1]]))
        else:
            w = mps.to_dense(st)[0][0]
            wg = got[0]
        np.testing.assert_allclose(np.log(wg) + ls, np.log(w) + lr[0], atol=1e-7)


def _group(d, p=0.1, batch=4, noise=None, p_dev=None):
    from paper_2402_04834_amd import _lib
    g = _lib.bbp_group()
    g.d, g.p, g.batch = d, p, batch
    if noise is not None:
        for k in range(4):
            g.noise[k] = noise[k]
    g.p_dev = p_dev
    return g


def test_group_validation(bbp):
    """bbp_workspace_size_groups validates every group (host only): noise probabilities, p, group count."""
    import ctypes as C
    from paper_2402_04834_amd import _lib
    h = _lib.lib()
    n = C.c_size_t()
    opts = bbp.default_opts(block=6, chi=32)

    def size(groups, o=opts):
        arr = (_lib.bbp_group * len(groups))(*groups)
        return h.bbp_workspace_size_groups(arr, len(groups), C.byref(o), C.byref(n))

    assert size([_group(9)]) == _lib.BBP_OK and n.value > 0
    one = n.value
    assert size([_group(9), _group(9)]) == _lib.BBP_OK and n.value >= 2 * one
    assert size([_group(9, noise=(0.9, 0.02, 0.06, 0.02))]) == _lib.BBP_OK
    assert size([_group(9, noise=(0.9, 0.02, 0.06, 0.03))]) == _lib.BBP_EINVAL          # does not sum to 1
    assert size([_group(9, noise=(0.0, 0.5, 0.5, 0.0))]) == _lib.BBP_EINVAL             # no identity weight
    assert size([_group(9, noise=(1.2, -0.1, -0.05, -0.05))]) == _lib.BBP_EINVAL        # negative entries
    assert size([_group(9, noise=(0.9, 0.02, 0.06, 0.02), p_dev=8)]) == _lib.BBP_EINVAL  # exclusive with p_dev
    assert size([_group(9, noise=(0.9, 0.02, 0.06, 0.02))], bbp.default_opts(block=6, chi=32, precision=1)) \
        == _lib.BBP_EUNSUPPORTED
    assert size([_group(9, p=1.5)]) == _lib.BBP_EINVAL
    assert size([_group(9)] * 9) == _lib.BBP_EINVAL                                     # at most 8 groups


def test_warm_start_host_side(bbp):
    """Parameter count of the network and workspace sizes; argument checks that precede any device work."""
    import ctypes as C
    from paper_2402_04834_amd import _lib, warm
    from oracle import warmnet
    assert warm.param_count() == warmnet.count() == 198648
    opts = bbp.default_opts(block=6, chi=32)
    small = warm.workspace_size(9, 4, opts, False)
    assert warm.workspace_size(9, 10000, opts, False) == warm.workspace_size(9, 512, opts, False) > small
    assert warm.workspace_size(9, 64, opts, True) > warm.workspace_size(9, 16, opts, True)
    h = _lib.lib()
    n = C.c_size_t()
    assert h.bbp_warm_workspace_size(9, 4, C.byref(bbp.default_opts(block=7, chi=32)), 0, C.byref(n)) \
        == _lib.BBP_EINVAL
    assert h.bbp_warm_predict(9, 0.1, None, None, 4, C.byref(opts), None, 1, None, None, 0, None) == _lib.BBP_EINVAL
    assert h.bbp_warm_adam(None, None, None, None, 1, C.c_float(1e-3), None) == _lib.BBP_EINVAL
    assert "NULL" in h.bbp_warm_last_error().decode() or "pointer" in h.bbp_warm_last_error().decode()
    # the committed weights have the network's shape
    assert warm.load().shape == (warm.param_count(),)


def test_bmps_and_gate_host_side(bbp):
    """Boundary-MPS workspace sizes (labels plus 20 KiB of FP64 state per grid row and coset network) and
    the argument checks that precede any device work; the gate option's range."""
    import ctypes as C
    from paper_2402_04834_amd import _lib
    h = _lib.lib()
    n = C.c_size_t()
    d, batch = 17, 8
    L = 2 * d - 1
    assert h.bbp_bmps_workspace_size(d, batch, 16, C.byref(n)) == _lib.BBP_OK
    label_bytes = -(-batch * 4 * L * L // 256) * 256
    # per row of each coset network: the compressed row [16][2][16] and the factor slot (32 reflection
    # vectors of 64 entries and their 32 coefficients), in doubles
    assert n.value == label_bytes + 4 * batch * L * (16 * 2 * 16 + 32 * 64 + 32) * 8
    assert h.bbp_bmps_workspace_size(d, batch, 17, C.byref(n)) == _lib.BBP_EINVAL     # chi above 16
    assert h.bbp_bmps_workspace_size(d, batch, 0, C.byref(n)) == _lib.BBP_EINVAL      # chi below 1
    assert h.bbp_bmps_workspace_size(1, batch, 16, C.byref(n)) == _lib.BBP_EINVAL     # d below 2
    assert h.bbp_bmps_workspace_size(d, -1, 16, C.byref(n)) == _lib.BBP_EINVAL        # negative batch
    # batch 0 is a no-op that touches no pointer; bad noise is refused before any launch
    assert h.bbp_bmps_decode_device(d, 0.1, None, None, None, 0, 16, None, 0, None, None, None, None, None) \
        == _lib.BBP_OK
    bad = (C.c_double * 4)(0.5, 0.2, 0.2, 0.2)
    assert h.bbp_bmps_decode_device(d, 0.1, None, bad, None, 0, 16, None, 0, None, None, None, None, None) \
        == _lib.BBP_EINVAL
    assert h.bbp_bmps_decode_device(d, 1.5, None, None, None, 0, 16, None, 0, None, None, None, None, None) \
        == _lib.BBP_EINVAL
    # the residual gate must be finite and non-negative
    assert h.bbp_workspace_size(d, batch, C.byref(bbp.default_opts(gate=1e-6)), C.byref(n)) == _lib.BBP_OK
    assert h.bbp_workspace_size(d, batch, C.byref(bbp.default_opts(gate=-1.0)), C.byref(n)) == _lib.BBP_EINVAL
    assert h.bbp_workspace_size(d, batch, C.byref(bbp.default_opts(gate=float("inf"))), C.byref(n)) \
        == _lib.BBP_EINVAL
