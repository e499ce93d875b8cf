"""CPU checks of the C ABI: the library loads, exports every function the
header declares, and rejects bad descriptors before touching the GPU."""
import ctypes
import os

import pytest

import workloads as W


@pytest.fixture(scope="module")
def vlb():
    from paper_2410_23802_amd import build as hb
    from paper_2410_23802_amd import vlb as v
    if not os.path.exists(v.LIB_PATH):
        hb.build()
    return v


def test_library_exports_header_symbols(vlb):
    names = vlb.header_functions()
    assert "vlb_step" in names and "vlb_create" in names
    L = vlb.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_descriptor_mirror_matches_header_field_order(vlb):
    """The ctypes mirror lists the header's struct members in order."""
    import re
    with open(vlb.HEADER) as fh:
        txt = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    body = re.search(r"typedef struct \{(.*?)\} vlb_domain_desc;", txt, re.S)
    decl = re.findall(r"\b([A-Za-z_]\w*)\s*(?:\[[^\]]*\])*\s*[,;]", body.group(1))
    assert decl == [f[0] for f in vlb.vlb_domain_desc._fields_]


def test_particle_mirror_matches_header(vlb):
    """The ctypes mirror of vlb_particle_desc lists the header's members in
    order, and the struct is ten doubles and two int32 (88 bytes)."""
    import re
    with open(vlb.HEADER) as fh:
        txt = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\} vlb_particle_desc;", txt)
    decl = re.findall(r"\b([A-Za-z_]\w*)\s*(?:\[[^\]]*\])*\s*[,;]", body.group(1))
    assert decl == [f[0] for f in vlb.vlb_particle_desc._fields_]
    assert ctypes.sizeof(vlb.vlb_particle_desc) == 88


@pytest.mark.parametrize("patch,msg", [
    ({"nx": 0}, "nx and ny"),
    ({"tau_f": 0.5}, "tau_f"),
    ({"face_flow": ["periodic", "wall", "periodic", "periodic"]}, "pairs"),
    ({"kmax": 0}, "kmax"),
    ({"lambda_f": -1.0}, "> 0"),
    ({"sigma_rule": 3}, "sigma_rule"),
    ({"fluid_gravity": 2}, "fluid_gravity"),
])
def test_create_rejects_bad_descriptor(vlb, patch, msg):
    d = W.domain(16, 16)
    d.update(patch)
    desc = vlb.make_domain_desc(d)
    h = ctypes.c_void_p()
    rc = vlb.lib().vlb_create(ctypes.byref(desc), None, ctypes.byref(h))
    assert rc == vlb.VLB_EINVAL
    assert h.value is None
    assert msg in vlb.vlb_last_error(None)


def test_create_rejects_unknown_precision(vlb):
    desc = vlb.make_domain_desc(W.domain(8, 8), precision=7)
    h = ctypes.c_void_p()
    assert vlb.lib().vlb_create(ctypes.byref(desc), None, ctypes.byref(h)) == vlb.VLB_EINVAL


def test_null_arguments(vlb):
    L = vlb.lib()
    assert L.vlb_create(None, None, None) == vlb.VLB_EINVAL
    assert L.vlb_step(None, 1) == vlb.VLB_EINVAL
    assert L.vlb_init(None) == vlb.VLB_EINVAL
    assert L.vlb_step_count(None) == -1
    L.vlb_destroy(None)


def test_batch_create_rejects_bad_arguments(vlb):
    """Checked before any device work: mixed precisions, too many particles
    in one domain, no domains."""
    L = vlb.lib()
    h = ctypes.c_void_p()
    descs = (vlb.vlb_domain_desc * 2)(vlb.make_domain_desc(W.domain(16, 16), "fp32"),
                                      vlb.make_domain_desc(W.domain(16, 16), "fp64"))
    counts = (ctypes.c_int32 * 2)(0, 0)
    assert L.vlb_batch_create(2, descs, counts, None, ctypes.byref(h)) == vlb.VLB_EINVAL
    assert "precision" in L.vlb_batch_last_error(None).decode()
    descs[1] = vlb.make_domain_desc(W.domain(16, 16), "fp32")
    counts[1] = 65
    parts = vlb.make_particles([W.particle(8, 8, 2)] * 65)
    assert L.vlb_batch_create(2, descs, counts, parts, ctypes.byref(h)) == vlb.VLB_EINVAL
    assert "0..64" in L.vlb_batch_last_error(None).decode()
    assert L.vlb_batch_create(0, descs, counts, parts, ctypes.byref(h)) == vlb.VLB_EINVAL
    assert h.value is None
    assert L.vlb_batch_step(None, 1) == vlb.VLB_EINVAL
    L.vlb_batch_destroy(None)


def test_library_carries_the_hash_of_its_sources(vlb):
    from paper_2410_23802_amd import build as hb
    assert vlb.lib().vlb_build_hash().decode() == hb.source_hash()


def test_stale_library_is_refused(vlb, monkeypatch):
    """A library built from other sources than those beside it does not
    load: the binding compares the hash the library carries with the
    sources'."""
    from paper_2410_23802_amd import build as hb
    saved = vlb._lib
    try:
        vlb._lib = None
        monkeypatch.setattr(hb, "source_hash", lambda: "0" * 16)
        with pytest.raises(vlb.VlbLibraryStale):
            vlb.lib()
    finally:
        vlb._lib = saved


def test_c_example_is_built_and_checks_its_arguments():
    """The plain C caller of the ABI is built beside the library; without
    its three arguments it prints its usage and exits 2 (before any GPU
    call)."""
    import subprocess
    from paper_2410_23802_amd import build as hb
    if not os.path.exists(hb.EXAMPLE):
        hb.build_example()
    r = subprocess.run([hb.EXAMPLE], capture_output=True, text=True,
                       timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
