"""The C ABI driven from plain C: paper_2410_23802_amd/examples/vlb_c_run,
a C program linked against libvlb.so with no Python or PyTorch in its
process (so on the HIP runtime of the system, not the one PyTorch ships),
steps a domain whose descriptor and particles the test writes as raw ABI
structs; its fields and particle states must equal, bit for bit, those of
the same run through the Python binding in this process."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("rho", "ux", "uy", "T", "fs", "dfs")


@pytest.fixture(scope="module")
def vlb():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2410_23802_amd import build as hb
    from paper_2410_23802_amd import vlb as v
    v.lib()  # fails loudly if the HIP library is missing or stale
    if not os.path.exists(hb.EXAMPLE):
        pytest.fail("the C example is not built (build() builds it)")
    return v


def run_c(vlb, tmp_path, d, ps, prec, nsteps):
    from paper_2410_23802_amd import build as hb
    desc = vlb.make_domain_desc(d, prec, None, None)
    arr = vlb.make_particles(ps)
    src, dst = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(src, "wb") as fh:
        fh.write(bytes(desc))
        fh.write(np.int32(len(ps)).tobytes())
        fh.write(bytes(arr)[:len(ps) * ctypes.sizeof(vlb.vlb_particle_desc)])
    env = {k: v for k, v in os.environ.items() if k != "LD_LIBRARY_PATH"}
    r = subprocess.run([hb.EXAMPLE, str(src), str(dst), str(nsteps)],
                       capture_output=True, text=True, timeout=120, env=env)
    print(r.stdout.strip(), flush=True)
    assert r.returncode == 0, r.stderr
    raw = dst.read_bytes()
    n = d["nx"] * d["ny"]
    fields = np.frombuffer(raw[:6 * n * 8], np.float64).reshape(6, d["ny"],
                                                                d["nx"])
    st = (vlb.vlb_particle_state * max(len(ps), 1)).from_buffer_copy(
        raw[6 * n * 8:].ljust(ctypes.sizeof(vlb.vlb_particle_state), b"\0"))
    return fields, st


@pytest.mark.parametrize("case,prec", [("scan", "fp64"), ("list", "fp64"),
                                       ("list", "fp32")])
def test_c_caller_matches_python_bit_for_bit(vlb, tmp_path, case, prec):
    if case == "scan":
        d, ps = W.c1_tiny()
        ps = [dict(ps[0], fixed=0, ux=0.004, uy=-0.002, omega=0.001,
                   rho_s=1.4)]
    else:
        d = W.walls(W.domain(300, 200, tau_f=0.7, lambda_f=0.05,
                             R_lambda=3.0, R_cv=1.5, gravity=(0.0, -4e-5),
                             beta=0.1, init_T=1.0, coll_range=2.0,
                             coll_stiff_pp=2e-3, coll_stiff_pw=4e-3))
        pts = W.rsa_disks(90, 4.0, (0.0, 0.0, 300.0, 200.0), 1.0, seed=4)
        ps = [W.particle(x, y, 4.0, rho_s=1.5, T_init=0.2) for x, y in pts]
    nsteps = 40
    print(f"case: C caller, {case} form, {prec}, {nsteps} steps", flush=True)
    fields, st = run_c(vlb, tmp_path, d, ps, prec, nsteps)
    dom = vlb.Domain(d, ps, prec).init().step(nsteps)
    for k, name in enumerate(FIELDS):
        assert np.array_equal(fields[k], dom.field(name)), name
    p = dom.particles()
    for k in range(len(ps)):
        for name in ("x", "y", "ux", "uy", "omega", "Fx", "Fy", "Tz",
                     "T_mean", "T_min", "E_solid"):
            assert getattr(st[k], name) == p[name][k], (k, name)
    dom.close()
