"""The C ABI library loads on a machine without a GPU and exports every
entry point include/nmdose.h, include/nmdose_nn.h, include/nmdose_ingest.h and
include/nmdose_probe.h
declare; calls without a device fail with a status instead of crashing."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f)
           for f in ("nmdose.h", "nmdose_nn.h", "nmdose_ingest.h", "nmdose_probe.h")]
LIB = os.path.join(ROOT, "paper_2111_11687_amd", "libnmdose.so")


def _declared():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"\b(nmd_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libnmdose.so is not built; run __graft_entry__.build()")
    return ctypes.CDLL(LIB)


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 38
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_the_header():
    from paper_2111_11687_amd import binding
    assert sorted(binding.EXPORTS) == _declared()


def test_default_options(lib):
    from paper_2111_11687_amd.binding import nmd_run_opts
    o = nmd_run_opts()
    lib.nmd_run_opts_default(ctypes.byref(o))
    assert o.photons_per_decay == 2 and o.process_mask == 7
    assert abs(o.photon_cutoff_mev - 0.010) < 1e-9 and o.source_kind == 0
    assert o.chunk == 0 and o.history_records is None


def test_struct_sizes_match_header():
    from paper_2111_11687_amd.binding import nmd_material, nmd_run_opts
    assert ctypes.sizeof(nmd_material) == 16
    # 5 u32/f32 + 6 floats + 3 u32, padded to 8, then one pointer
    assert ctypes.sizeof(nmd_run_opts) == 64


def test_ingest_struct_layout_matches_the_c_compiler(tmp_path):
    """sizeof and field offsets of nmd_grid and nmd_ct_table as gcc lays out
    the header, against the binding's ctypes structures."""
    import subprocess
    from paper_2111_11687_amd.binding import nmd_ct_table, nmd_grid
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "nmdose_ingest.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(nmd_grid), offsetof(nmd_grid, spacing_mm),
         offsetof(nmd_grid, origin_mm), sizeof(nmd_ct_table));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(nmd_ct_table, hu),
         offsetof(nmd_ct_table, density), offsetof(nmd_ct_table, n_materials),
         offsetof(nmd_ct_table, hu_threshold), offsetof(nmd_ct_table, density_min),
         offsetof(nmd_ct_table, density_width), offsetof(nmd_ct_table, levels));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    c = [int(x) for x in out]
    py = [ctypes.sizeof(nmd_grid), nmd_grid.spacing_mm.offset, nmd_grid.origin_mm.offset,
          ctypes.sizeof(nmd_ct_table), nmd_ct_table.hu.offset, nmd_ct_table.density.offset,
          nmd_ct_table.n_materials.offset, nmd_ct_table.hu_threshold.offset,
          nmd_ct_table.density_min.offset, nmd_ct_table.density_width.offset,
          nmd_ct_table.levels.offset]
    assert c == py


def test_calls_without_a_device_fail_cleanly(lib):
    lib.nmd_last_error.restype = ctypes.c_char_p
    assert lib.nmd_last_error(None) == b"no context"
    h = ctypes.c_void_p()
    st = lib.nmd_create(ctypes.byref(h), 0, None)
    if st == 0:  # a GPU is present: the context is valid, release it
        lib.nmd_destroy(h)
    else:
        assert st == -1 and not h.value
    assert lib.nmd_run_histories(None, 0, 10, 1, None) == -1
    assert lib.nmd_set_activity(None, 0, None, ctypes.c_double(0.0)) == -1
