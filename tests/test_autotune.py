"""Candidate enumeration of the autotuner (host logic): every candidate
satisfies the library's own validation, is a multiple of dz dividing the
spans, and is the longest such long step for its block size and halo."""
import ctypes as C

from workloads import WORKLOADS, dm_map


def test_candidates_are_valid_and_maximal():
    from paper_1101_0086_amd import _lib as L
    from paper_1101_0086_amd.autotune import HALO_RULE, candidates
    w = WORKLOADS["wdm8_n262144_f32"]
    dz = 1.25e-4
    cands = candidates(w.grid.n, w.grid.dt, w.dmmap, dz, w.mpa.omega_band, shifted=False)
    # halos of 64 and 128 samples cannot take even one dz inside the halo rule
    assert [(c.block, c.halo) for c in cands] == [(1024, 256), (1024, 384), (2048, 256), (2048, 512), (2048, 768),
                                                  (4096, 512), (4096, 1024), (4096, 1536),
                                                  (8192, 1024), (8192, 2048), (8192, 3072),
                                                  (16384, 2048), (16384, 4096), (16384, 6144),
                                                  (32768, 4096), (32768, 8192), (32768, 12288)]
    rate = max(abs(b2) * w.mpa.omega_band + 0.5 * abs(b3) * w.mpa.omega_band ** 2
               for b2, b3 in zip(w.dmmap.beta2, w.dmmap.beta3))
    m = L.MapStruct(w.dmmap)
    for c in cands:
        assert abs(c.L - c.M * dz) < 1e-15 and c.halo in (c.block // 8, c.block // 4, 3 * c.block // 8)
        p = L.make_params(w.grid.n, w.grid.dt, c.L, c.M, 2, c.block, c.halo, 0, w.mpa.omega_band)
        assert L.lib().mpa_plan_validate(C.byref(p), C.byref(m.s)) == L.MPA_OK
        # the next admissible multiple of dz breaks the halo rule
        nxt = [k for k in range(c.M + 1, 4001) if 4000 % k == 0][0]
        assert rate * nxt * dz > HALO_RULE * c.halo * w.grid.dt
    # the 4096-block, 512-halo candidate has the benchmark's long step (the
    # benchmark takes M = 4 nodes per long step, dz = L / 4, instead of
    # dz = L / 2); the wider halo admits a longer one
    by = {(c.block, c.halo): c for c in cands}
    assert by[(4096, 512)].L == w.mpa.L
    assert by[(4096, 1024)].L > w.mpa.L


def test_no_candidate_when_halo_rule_cannot_hold():
    from paper_1101_0086_amd.autotune import candidates
    dmm = dm_map(beta3=0.1)
    assert candidates(1 << 16, 10 / 1024, dmm, 0.25, 145.0) == []


def test_shifted_candidates_are_valid_maximal_and_longer():
    """With windows shifted by the middle of the band's group-delay range,
    every candidate passes the library's validation with its shift, the next
    admissible long step does not, and no long step is shorter than the
    unshifted candidate's."""
    from paper_1101_0086_amd import _lib as L
    from paper_1101_0086_amd.autotune import candidates, window_shift
    w = WORKLOADS["wdm32_n4194304_f32"]
    dz = w.mpa.L / w.mpa.M
    plain = {(c.block, c.halo): c for c in candidates(w.grid.n, w.grid.dt, w.dmmap, dz, w.mpa.omega_band,
                                                        shifted=False)}
    cands = candidates(w.grid.n, w.grid.dt, w.dmmap, dz, w.mpa.omega_band)
    m = L.MapStruct(w.dmmap)
    longer = 0
    for c in cands:
        assert c.shift == window_shift(w.dmmap, w.mpa.omega_band, c.L, w.grid.dt, c.halo)
        p = L.make_params(w.grid.n, w.grid.dt, c.L, c.M, 2, c.block, c.halo, 0, w.mpa.omega_band, shift=c.shift)
        assert L.lib().mpa_plan_validate(C.byref(p), C.byref(m.s)) == L.MPA_OK
        nxt = [k for k in range(c.M + 1, 64001) if 64000 % k == 0][0]
        sh = window_shift(w.dmmap, w.mpa.omega_band, nxt * dz, w.grid.dt, c.halo)
        p = L.make_params(w.grid.n, w.grid.dt, nxt * dz, nxt, 2, c.block, c.halo, 0, w.mpa.omega_band, shift=sh)
        assert L.lib().mpa_plan_validate(C.byref(p), C.byref(m.s)) == L.MPA_EHALO
        base = plain.get((c.block, c.halo))
        assert base is None or c.L >= base.L
        longer += base is None or c.L > base.L
    assert longer >= 3
    # the 4096-block, 512-halo candidate takes two dz per long step instead of one,
    # and the 1024-halo one four (the workload's configuration)
    by = {(c.block, c.halo): c for c in cands}
    assert by[(4096, 512)].M == 2 and by[(4096, 1024)].M == w.mpa.M and by[(4096, 1024)].shift == w.mpa.shift
