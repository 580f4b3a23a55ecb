"""The measurement probes behind the roofline (include/nmdose_probe.h):
each runs and reports a positive launch time or rate, and refuses
arguments outside its documented range."""
import pytest

from paper_2111_11687_amd import binding as B

pytestmark = pytest.mark.gpu


def test_lds_probe_patterns_and_validation(engine):
    for write in (False, True):
        for p in B.LDS_PATTERNS:
            assert B.nmd_probe_lds(engine.ctx, p, write, 16, 8) > 0.0
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_probe_lds(engine.ctx, len(B.LDS_PATTERNS), False, 16, 8)
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_probe_lds(engine.ctx, 0, False, 0, 8)
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_probe_lds(engine.ctx, 0, False, 16, 65537)


def test_unit_and_ceiling_probes_run(engine):
    for k in B.UNITS:
        assert B.nmd_probe_unit(engine.ctx, k, 4, 16) > 0.0
    rate, ms = B.nmd_probe_ceiling(engine.ctx, "copy", 1 << 20, 2)
    assert rate > 0.0 and ms > 0.0
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_probe_ceiling(engine.ctx, "copy", 3 << 20, 2)
    with pytest.raises(B.NmdError, match="NMD_E_INVALID"):
        B.nmd_probe_unit(engine.ctx, len(B.UNITS), 4, 16)
