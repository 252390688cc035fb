"""The parallel oracle driver used by the full-size GPU parity tests gives
exactly what the in-process oracle gives (digests of the same bytes, rz
records with list-wide peak indices)."""
import numpy as np

import oracle
import oracle_pool
import synth


def test_event_digests_equal_in_process_oracle():
    name = "c4_batch_4096"
    spec = synth.grid_spec(name)
    spec.update(n_qpt=32, n_phi=64)
    got = oracle_pool.event_digests(name, spec, [0, 5, 17])
    tab = oracle.Tables(spec)
    for e in (0, 5, 17):
        ev = synth.gen_batch(name, 1, first_event=e)
        A, pk, _ = oracle.run_event(tab, ev.layer, ev.phi, with_rz=False)
        assert got[e][:2] == (oracle_pool.digest(A), oracle_pool.digest(pk.astype(oracle_pool.PEAK_DTYPE)))
    assert oracle_pool.digest(np.zeros(4, np.uint16)) != oracle_pool.digest(np.ones(4, np.uint16))


def test_rz_records_in_chunks_equal_one_call():
    name = "c2_single_1ktrk_rz"
    spec = synth.grid_spec(name)
    spec.update(n_qpt=64, n_phi=64)
    ev = synth.gen_config(name)
    tab = oracle.Tables(spec)
    A, pk, rz = oracle.run_event(tab, ev.layer, ev.phi, ev.z)
    got = oracle_pool.rz_records(name, spec, pk, chunk=97)
    np.testing.assert_array_equal(got, rz.astype(oracle_pool.RZ_DTYPE))
