"""fem_batch_get_contact_patch_noalloc (the contact patch staged in the
library's static device scratch, for callers that cannot allocate) against
fem_batch_get_contact_patch (its batch-allocated staging), through the C ABI:
two calls in a row, the second on a job of a smaller mesh, each compared
entry by entry (same kernel on the same state: identical results), plus the
documented errors."""
import numpy as np
import pytest

from paper_2103_16747_amd import fem, workload as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def short_job(mesh, seed, steps=4, depth=0.8e-3):
    """The seed's indenter pressed `depth` in `steps` load steps."""
    ind = W.seat_on_mesh(W.random_indentation(seed), mesh)
    return W.Indentation(ind.kind, ind.shape, ind.R, ind.c0, ind.direction, depth, steps, ind.k_penalty, seed=seed)


def noalloc_patch(batch, job, cap):
    ids = np.full(cap, -1, dtype=np.int32)
    f = np.full((cap, 3), np.nan)
    phi = np.full(cap, np.nan)
    Ft = np.full(3, np.nan)
    n = batch.contact_patch_noalloc(job, ids, f, phi, Ft)
    return ids[:n], f[:n], phi[:n], Ft


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_contact_patch_matches_allocating_call(precision):
    big, small = W.fingertip_mesh(50000), W.fingertip_mesh(5000)
    batch = fem.FemBatch(4, precision)
    mb = batch.add_mesh(big.X, big.tets, big.fixed)
    ms = batch.add_mesh(small.X, small.tets, small.fixed)
    jb = batch.add_job(mb, short_job(big, 3000))
    js = batch.add_job(ms, short_job(small, 3002))
    assert batch.run() == 0
    cases = ((jb, "50k-tet mesh"), (js, "5k-tet mesh"))
    for job, what in cases:
        say("case", precision, what)
        ids_r, f_r, phi_r, F_r = batch.contact_patch(job)
        assert len(ids_r) > 3, "the job should end in contact over several nodes"
        ids, f, phi, Ft = noalloc_patch(batch, job, len(ids_r) + 8)
        say(f"{precision} {what}: {len(ids)} contact nodes, resultant {Ft}")
        np.testing.assert_array_equal(ids, ids_r)
        np.testing.assert_array_equal(f, f_r)
        np.testing.assert_array_equal(phi, phi_r)
        np.testing.assert_array_equal(Ft, F_r)
        assert np.all(np.diff(ids) > 0)
    # count-only query, then a capacity below the count
    Ft = np.zeros(3)
    n = batch.contact_patch_noalloc(jb, None, None, None, Ft)
    assert n == len(batch.contact_patch(jb)[0])
    with pytest.raises(fem.FemError) as e:
        noalloc_patch(batch, jb, n - 1)
    assert e.value.code == fem.FEM_E_BUFFER
    # f without ids is refused (the ids order the entries)
    with pytest.raises(fem.FemError) as e:
        batch.contact_patch_noalloc(jb, None, np.zeros((n, 3)), None, Ft)
    assert e.value.code == fem.FEM_E_INVALID
    # a job added since the last run: the launch tables are stale
    batch.add_job(ms, short_job(small, 3005))
    with pytest.raises(fem.FemError) as e:
        noalloc_patch(batch, js, n + 8)
    assert e.value.code == fem.FEM_E_STATE
    batch.close()
