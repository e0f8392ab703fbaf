"""Host replay of the relaxation kernels' index arithmetic (no GPU needed).

``rve_check_indexing`` packs a batch exactly as ``rve_batch_create`` does and,
for every RVE and every register-resident kernel build whose slots hold it,
bounds every index the build forms: the packed fiber ends against the LDS
position array (free nodes plus the zero slot), the register-held incidence
codes and the CSR overflow reads against the LDS force array (fibers plus
the zero slot), the code's end sign and fiber bits, the workgroup's LDS bytes
against 160 KB; the streamed engine's workspace offsets; and the packing's
incidence lists (every fiber end listed once, with its sign).  The kernels
form these indices with the same helper functions (``res_pack_ends``,
``res_inc_code``, ``res_code_fiber``) that the replay calls.
"""
import numpy as np
import pytest

from paper_2306_09427_amd import binding as rb
from paper_2306_09427_amd import synth

pytestmark = pytest.mark.skipif(not __import__("os").path.exists(rb.LIB_PATH), reason="library not built")


@pytest.fixture(scope="module")
def cfg2():
    return synth.make_config_batch(2, idx=np.arange(64), workers=4)[0]


@pytest.mark.parametrize("precision", [rb.FP64, rb.MIXED])
def test_config2_networks_index_in_bounds(cfg2, precision):
    rb.check_indexing(cfg2, precision)


@pytest.mark.parametrize("precision", [rb.FP64, rb.MIXED])
def test_config5_networks_index_in_bounds(precision):
    # the lognormal size mix of the FE2 workload: RVEs from 100 to 3000 seeds,
    # below and above every resident capacity
    idx = [0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144]
    batch = synth.make_config_batch(5, idx=idx, workers=4)[0]
    nfib = np.diff(batch.fib_off)
    assert nfib.max() > 4096 and nfib.min() < 2048
    rb.check_indexing(batch, precision)


def test_small_and_degenerate_networks_index_in_bounds():
    nets = [synth.lattice_network(n) for n in (2, 3, 5)]
    nets.append(synth.single_fiber_network([0.0, 0.3, 0.4], [1.0, 0.6, 0.5]))
    nets.append(synth.chain_network([[0.0, 0.5, 0.5], [0.3, 0.6, 0.5], [0.6, 0.4, 0.5], [1.0, 0.5, 0.5]]))
    # a free hub of degree 12 (incidences beyond the register-held four)
    rng = np.random.default_rng(3)
    ends = rng.random((12, 3))
    ends[np.arange(12), np.arange(12) % 3] = np.arange(12) % 2
    X = np.vstack([[0.5, 0.5, 0.5], ends])
    fib = np.array([[0, k + 1] for k in range(12)], np.int32)
    nets.append(synth.Network(X, np.r_[0, np.ones(12)].astype(np.uint8), fib))
    batch = synth.pack(nets)
    for p in (rb.FP64, rb.MIXED):
        rb.check_indexing(batch, p)


def test_prestressed_rest_lengths_index_in_bounds(cfg2):
    L0 = np.full(int(cfg2.fib_off[-1]), 0.05)
    rb.check_indexing(cfg2, rb.MIXED, L0=L0)


def test_planted_lds_mistake_is_reported(cfg2):
    """With the LDS position array assumed one entry short, the replay must
    find the fiber whose boundary end reads the zero slot."""
    with pytest.raises(rb.RVEError) as e:
        rb.check_indexing(cfg2, rb.MIXED, plant=1)
    assert "outside the LDS array" in str(e.value)


@pytest.mark.parametrize("precision", [rb.FP64, rb.MIXED])
def test_largest_rves_index_in_bounds(precision):
    """The largest RVEs of the FE2 workload (above 12288 free nodes: the
    incidence engine's global mode, node state in [NFREE + R] arrays)."""
    seeds = np.array([synth.seed_count(5, r) for r in range(8192)])
    batch = synth.make_config_batch(5, idx=np.sort(np.argsort(seeds)[-2:]), workers=2)[0]
    nfree = [int((batch.is_bnd[batch.node_off[r]:batch.node_off[r + 1]] == 0).sum()) for r in range(batch.n_rve)]
    assert max(nfree) > 12288
    rb.check_indexing(batch, precision)


def test_planted_incidence_record_mistake_is_reported(cfg2):
    """With one incidence record naming the wrong other end, the replay of
    the incidence engine's tables must report it."""
    with pytest.raises(rb.RVEError) as e:
        rb.check_indexing(cfg2, rb.MIXED, plant=2)
    assert "wrong other end" in str(e.value)


@pytest.mark.parametrize("precision", [rb.FP64, rb.MIXED])
def test_large_rve_team_partitions_index_in_bounds(precision):
    """2000-seed RVEs (the large-RVE workload) take the team engine: the
    replay checks each part's tables (every free node owned once, every
    fiber of an owned node in the part, local ends naming the true ends,
    incidence codes naming the node's own fibers with its end's sign, halo
    exchange slots equal to the owners', capacities and LDS)."""
    batch = synth.make_config_batch(3, idx=[0, 1], workers=2)[0]
    assert np.diff(batch.fib_off).min() > 6144
    rb.check_indexing(batch, precision)
