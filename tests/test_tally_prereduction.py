"""Why the transport tally has no cross-lane pre-reduction before its FP64
atomics.  The history-by-history merge already combines a history's own
deposits per voxel.  Across lanes, a wave-level pre-reduction would combine
deposits of different histories that end in the same pass and land in the
same voxel.  With m merged deposits per pass spread over voxels with
probabilities p_v, the expected number of such pairs is
m (m - 1) / 2 * sum_v p_v^2.  This test measures sum_v p_v^2 on the patient
phantom from an oracle tally and bounds the pairs: below 0.05 % of the
deposits of a pass, however many of a wave's 64 lanes end together, so a
cross-lane match would cost a wave-wide comparison on every pass to save
fewer than one atomic in 2000."""
import numpy as np

from paper_2111_11687_amd import phantoms as P


def test_same_voxel_deposits_across_lanes_are_rare(orc):
    prob = P.patient_phantom()
    ph = orc.Phantom(prob.density, prob.material, [m[0] for m in prob.materials],
                     [m[1] for m in prob.materials], prob.voxel_cm, label=prob.label,
                     n_organs=prob.n_organs, activity=prob.activity)
    n = 1_000_000
    tal, _ = orc.run(ph, n, 91, tracking=orc.TRACK_WOODCOCK)
    s, s2 = tal.S.reshape(-1), tal.S2.reshape(-1)
    merged = tal.stats["merged"] / n
    # two weightings of p_v: by energy, and by the deposit count S^2 / S2
    # (exact when a voxel's deposits are equal)
    pe = s / s.sum()
    hit = s > 0
    cnt = np.zeros_like(s)
    cnt[hit] = s[hit] ** 2 / s2[hit]
    pc = cnt / cnt.sum()
    for p in (pe, pc):
        m = 64 * merged  # every lane of the wave ending its history at once
        pairs = m * (m - 1) / 2 * float((p * p).sum())
        assert pairs / m < 5e-4
