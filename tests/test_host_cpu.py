"""CPU tests of the library's host side: exported symbols, the poset / layout builder
(cross-checked against the oracle's own poset) and argument validation.  No device
compute is called here."""
import re

import numpy as np
import pytest

import lrh_workloads as W
from oracle import lrh_oracle as O
from paper_2609_40336_amd import lrh

from conftest import ROOT


def header_functions():
    src = open(f"{ROOT}/include/lrh.h").read()
    return sorted(set(re.findall(r"^(?:lrh_status|void|const char\*)\s+(lrh_\w+)\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = lrh.load()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lrh.EXPORTS)


def _two_level(d):
    return W.with_tops(d, list(d.tops()), two_level=True)


PROBLEMS = [
    lambda: W.workload_c1(),
    lambda: W.heisenberg_square(4),
    lambda: W.random_chain(9, seed=1, top_len=4, subintervals=True),
    lambda: W.random_chain(8, seed=2, top_len=6, subintervals=True),
    lambda: W.tfim_plaquette_batch([3, 5, 4], [0.5, 1.0, 3.0]),
    lambda: W.xxz_triangular(4, 0.5, seed=5),
    lambda: W.classical_ising_tree(9, 3),
    lambda: W.interval_chain_gue(12, 5, 0.1, seed=3),
    lambda: W.interval_chain_gue(12, 5, 0.1, seed=3, two_level=True),
    lambda: W.random_chain(9, seed=1, top_len=2, two_level=True),
    lambda: _two_level(W.classical_ising_tree(9, 3)),
    lambda: _two_level(W.tfim_plaquette_batch([3, 5, 4], [0.5, 1.0, 3.0])),
    lambda: W.spin1_chain(6),
    lambda: W.spin1_chain(7, top_len=3, subintervals=True, dm=0.2),
    lambda: W.spin1_chain(7, top_len=3, two_level=True),
]


@pytest.mark.parametrize("maker", PROBLEMS)
def test_host_poset_matches_oracle(maker):
    d = maker()
    P = lrh.Problem(d, -1)
    R = O.Relaxation(d)
    assert sorted(P.clusters) == sorted(R.clusters)
    assert set(P.message_keys()) == {(R.clusters[e], R.clusters[f]) for (e, f) in R.msgs}
    assert P.n_msgs == R.n_msgs
    assert P.Lambda == pytest.approx(R.Lambda)
    assert P.Gamma == pytest.approx(R.Gamma)
    # clusters are grouped by instance, every per-instance range is contiguous
    inst = P.cluster_instance
    assert np.all(np.diff(inst) >= 0)
    # layout: buckets partition nu_len
    tot = sum(b["M"] * b["comps"] for b in P.buckets)
    assert tot == P.nu_len


def test_layout_round_trip():
    d = W.random_chain(7, seed=4, top_len=3, subintervals=True)
    P = lrh.Problem(d, -1)
    R = O.Relaxation(d)
    mats = R.to_pairs(R.draw(3, 1.0))
    v = P.from_dense_np(mats)
    back = P.to_dense(v)
    for k in mats:
        np.testing.assert_array_equal(back[k], mats[k])


def _expect(code, fn):
    with pytest.raises(lrh.LrhError) as e:
        fn()
    assert e.value.code == code, str(e.value)


def test_validation_errors():
    good = W.tfim_chain(4, 1.0, 0.5)
    # non-Hermitian term
    bad = W.tfim_chain(4, 1.0, 0.5)
    bad.term_im = np.zeros_like(bad.term_re)
    bad.term_im[1] = 0.3
    _expect(1, lambda: lrh.Problem(bad, -1))
    # site dimension 4 (spin-1/2 and spin-1 sites only); a spin-1 cluster above 64 dimensions
    d4 = W.tfim_chain(4, 1.0, 0.5)
    d4.site_dim = d4.site_dim.copy()
    d4.site_dim[0] = 4
    _expect(2, lambda: lrh.Problem(d4, -1))
    _expect(2, lambda: lrh.Problem(W.spin1_chain(6, top_len=4, subintervals=True), -1))
    # cluster spanning two instances
    sp = W.tfim_chain(4, 1.0, 0.5)
    sp.site_instance = np.array([0, 0, 1, 1], dtype=np.int32)
    sp.n_instances = 2
    _expect(1, lambda: lrh.Problem(sp, -1))
    # 9-site cluster (D_e = 512)
    big = W.with_tops(W.tfim_chain(10, 1.0, 0.5), [tuple(range(9))])
    _expect(2, lambda: lrh.Problem(big, -1))
    # unsorted top cluster
    uns = W.tfim_chain(4, 1.0, 0.5)
    uns.top_sites = uns.top_sites.copy()
    uns.top_sites[0], uns.top_sites[1] = uns.top_sites[1], uns.top_sites[0]
    _expect(1, lambda: lrh.Problem(uns, -1))
    # two-level family: with the interval closure, and with a term outside every top
    both = W.random_chain(6, seed=1, top_len=3, two_level=True)
    both.subintervals = True
    _expect(1, lambda: lrh.Problem(both, -1))
    orphan = W.with_tops(W.tfim_chain(5, 1.0, 0.5), [(0, 1, 2), (1, 2, 3)], two_level=True)
    _expect(1, lambda: lrh.Problem(orphan, -1))
    # 2 x 3 plaquettes on the 4 x 4 torus overlap in 3 and in 4 sites: children of one cluster
    # with different dimensions are not supported
    _expect(2, lambda: lrh.Problem(_two_level(W.tfim_rect_plaquettes(4, 1.0)), -1))
    # compute on a host-only problem
    P = lrh.Problem(good, -1)
    _expect(1, lambda: lrh._check(lrh.load().lrh_certify(P.h, 8, 0, 8, 8, None, None)))
    _expect(1, lambda: lrh._check(lrh.load().lrh_time_messages(P.h, 8, 8, 0, 1.0, 1, 8, None)))
    _expect(1, lambda: lrh._check(lrh.load().lrh_time_messages(P.h, 8, 8, 0, 1.0, 0, 8, None)))
    _expect(1, lambda: lrh._check(lrh.load().lrh_time_messages(P.h, None, 8, 0, 1.0, 1, 8, None)))


def test_batch_scaled_instances_are_scaled_copies():
    """The batching helper used by the iterations-to-eps experiment: instance i of the batch is
    descs[i] with every term times scales[i] (checked on the oracle's Anderson bound Q(0), which
    is positively homogeneous in H)."""
    import lrh_workloads as W
    from oracle import lrh_oracle as O
    descs = [W.heisenberg_chain(5, field_x=0.5), W.tfim_chain(4, 1.0, 1.0, complex_storage=False),
             W.random_chain(4, seed=7)]
    scales = [2.0, 0.25, 3.0]
    Rb = O.Relaxation(W.batch_scaled(descs, scales))
    qb = Rb.Q(Rb.zeros())
    for i, (d, s) in enumerate(zip(descs, scales)):
        R = O.Relaxation(d)
        assert abs(qb[i] - s * R.Q(R.zeros())[0]) <= 1e-12 * max(1.0, abs(qb[i]))


def test_one_hip_runtime_and_versions_recorded():
    """torch is imported before the library, so the process maps exactly one libamdhip64 (two
    runtimes under one soname crash torch's own launches); the library names the HIP headers it
    was compiled against, torch the release it ships."""
    info = lrh.runtime_info()
    assert len(info["mapped"]) == 1, info
    assert info["library"].startswith("HIP headers ") and "gfx950" in info["library"]
    assert info["torch_hip"]
    print("HIP runtime:", info)


def test_settings_calls_and_defaults_on_host_problem():
    """Settings calls validate their arguments; the slab limit accepts 0 (default) and positive
    caps.  Compute calls on a host-only problem are rejected before any default is applied."""
    P = lrh.Problem(W.tfim_chain(4, 1.0, 0.5), -1)
    P.set_slab_limit(2)
    P.set_slab_limit(0)
    _expect(1, lambda: P.set_slab_limit(-1))
    P.set_jacobi(30, 0.0)
    _expect(1, lambda: P.set_jacobi(-1, 0.0))
    st = lrh.NesterovState()
    st.k, st.theta, st.beta, st.L = 0, 1.0, 2.0, 0.0
    _expect(1, lambda: lrh._check(lrh.load().lrh_step_nesterov(P.h, 8, 8, lrh.C.byref(st), 1, 0, None)))


def test_certify_method_and_fallback_counter_validation():
    """The certification switch accepts methods 0..3 on any problem; the fallback counter needs a
    device problem and a count pointer."""
    P = lrh.Problem(W.tfim_chain(4, 1.0, 0.5), -1)
    for m in (0, 1, 2, 3, 0):
        P.set_certify_method(m)
    _expect(1, lambda: P.set_certify_method(-1))
    _expect(1, lambda: P.set_certify_method(4))
    n = lrh.C.c_int64(0)
    _expect(1, lambda: lrh._check(lrh.load().lrh_certify_fallbacks(P.h, None, lrh.C.byref(n))))
    _expect(1, lambda: lrh._check(lrh.load().lrh_certify_fallbacks(P.h, None, None)))
    _expect(1, lambda: lrh._check(lrh.load().lrh_set_certify_method(None, 0)))
