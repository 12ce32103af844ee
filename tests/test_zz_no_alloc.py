"""qmc_observe_noalloc (the estimators for callers that cannot allocate) through the C ABI against
qmc_observe on the same stores: integer numerators bit for bit, FP64 values to a few ulps (the
same operations in the same order, on the device instead of the host).  Two calls in a row, the
second with a smaller input (fewer qubits, replicas, keys and observables), share the library's
one scratch array; an input beyond its limits is refused before anything runs."""
import numpy as np
import pytest

from paper_2502_18929_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_18929_amd import binding
    binding.lib()
    return binding


def _device_store(g, n, R):
    """A context's store, all replicas, as device tensors of composite keys and (re, im)."""
    import torch
    ks, vs = [], []
    for r in range(R):
        k, a, b = g.export(r)
        ks.append((np.uint64(r) << np.uint64(2 * n)) | k)
        vs.append(np.stack([a, b], axis=1))
    keys = np.concatenate(ks).astype(np.uint64)
    vals = np.ascontiguousarray(np.concatenate(vs).astype(np.int32))
    return (torch.from_numpy(keys.view(np.int64)).cuda(), torch.from_numpy(vals).cuda(),
            len(keys))


def _same(got, ref, R, npl):
    for f in ("n_occ", "n_tot", "ndiag", "pauli", "eps2"):
        assert np.array_equal(got[f], ref[f]), f
    assert got["eps2_int"] == ref["eps2_int"]
    for f in ("trace", "theta", "pauli_val", "fidelity", "eps"):
        np.testing.assert_allclose(got[f], ref[f], rtol=1e-13, atol=1e-15, err_msg=f)
    assert got["n_occ"].shape == (R,) and got["pauli"].shape == (R, npl, 2)


def test_observe_noalloc_matches_observe_twice(B):
    import torch
    # first call: ghz4 after its 400 steps, 4 replicas, Pauli observables and the GHZ fidelity
    w = W.config_ghz4()
    g = B.QMC.from_workload(w, store_capacity=256, spawn_capacity=4096)
    g.step(w.s, w.gamma)
    pauli = [(x, z) for _, x, z, _ in w.pauli_obs] + [(3, 5), (15, 15), (0, 0), (6, 9)]
    ref = g.observe(pauli=pauli, psi=w.psi, want_eps=True)
    keys, vals, m = _device_store(g, w.n, w.n_replicas)
    nd0 = [w.walker_target] * w.n_replicas
    got = B.observe_noalloc(w.n, w.n_replicas, keys, vals, nd0, pauli=pauli, psi=w.psi,
                            want_eps=True)
    torch.cuda.synchronize()
    _same(got, ref, w.n_replicas, len(pauli))
    assert int(got["n_occ"].sum()) == m
    g.close()
    # second call, smaller: DD on 3 qubits, 2 replicas, one observable, a one-element |psi>
    w2 = W.dd(n=3, n_replicas=2, walker_target=5000, nsteps=150, seed=4)
    g2 = B.QMC.from_workload(w2, store_capacity=64, spawn_capacity=1024)
    g2.run_workload(w2, 0, 150)
    pauli2 = [(1, 0)]
    ref2 = g2.observe(pauli=pauli2, psi=w2.psi, want_eps=True)
    keys2, vals2, m2 = _device_store(g2, w2.n, w2.n_replicas)
    assert m2 < m
    got2 = B.observe_noalloc(w2.n, w2.n_replicas, keys2, vals2, [w2.walker_target] * 2,
                             pauli=pauli2, psi=w2.psi, want_eps=True)
    _same(got2, ref2, w2.n_replicas, 1)
    g2.close()


def test_observe_noalloc_refuses_beyond_its_limits(B):
    import torch
    keys = torch.zeros(1, dtype=torch.int64, device="cuda")
    vals = torch.ones((1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(B.QMCError) as e:      # more replicas than the scratch holds
        B.observe_noalloc(4, 300, keys, vals, [1] * 300)
    assert e.value.code == B.QMC_ERR_ARG
    with pytest.raises(B.QMCError) as e:      # a Pauli mask outside n bits
        B.observe_noalloc(4, 1, keys, vals, [1], pauli=[(1 << 4, 0)])
    assert e.value.code == B.QMC_ERR_ARG
    with pytest.raises(B.QMCError) as e:      # |psi|^2 x replicas beyond the lookup area
        B.observe_noalloc(6, 64, keys, vals, [1] * 64, psi=[(i, 0.1) for i in range(32)])
    assert e.value.code == B.QMC_ERR_ARG
