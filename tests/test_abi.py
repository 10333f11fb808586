"""The C ABI library loads and exports every entry point include/pa.h
declares; argument checks that need no device are exercised on the CPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pa.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pa_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_hot_path():
    names = _declared()
    for n in ("pa_init", "pa_sweep", "pa_resample", "pa_observables",
              "pa_free_energy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2006_00561_amd import binding
    lib = binding.lib()
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_and_validation_without_device():
    from paper_2006_00561_amd import binding as b
    lib = b.lib()
    assert lib.pa_strerror(b.PA_ECAPACITY).decode().startswith("population")
    h = C.c_void_p()
    for L, R, layout, rpl in ((3, 10, 0, 0), (130, 10, 0, 0), (16, 0, 0, 0),
                              (16, 10, 7, 0), (16, 10, 0, 3), (12, 10, 0, 8),
                              (128, 10, 0, 1)):
        cfg = b.pa_config()
        cfg.L, cfg.R_target, cfg.layout, cfg.rows_per_lane = L, R, layout, rpl
        assert lib.pa_init(C.byref(cfg), C.byref(h)) == b.PA_EINVAL
        assert not h.value
    cfg = b.pa_config()
    cfg.L, cfg.R_target, cfg.model = 8, 10, b.PA_PMJ   # +-J without couplings
    assert lib.pa_init(C.byref(cfg), C.byref(h)) == b.PA_EINVAL
    cfg = b.pa_config()
    cfg.L, cfg.R_target, cfg.resampling = 8, 10, 5      # no such law
    assert lib.pa_init(C.byref(cfg), C.byref(h)) == b.PA_EINVAL
    cfg = b.pa_config()
    cfg.L, cfg.R_target, cfg.rng_mode = 8, 10, 2        # no such stream
    assert lib.pa_init(C.byref(cfg), C.byref(h)) == b.PA_EINVAL
    cfg = b.pa_config()                                 # Potts: word mode only
    cfg.L, cfg.R_target, cfg.model, cfg.q = 8, 10, b.PA_POTTS, 3
    cfg.rng_mode = b.PA_RNG_PLANES
    assert lib.pa_init(C.byref(cfg), C.byref(h)) == b.PA_EINVAL
    assert not h.value
    # the batch takes the nearest-integer law only
    cfg = b.pa_config()
    cfg.L, cfg.R_target, cfg.resampling = 8, 10, b.PA_POISSON
    bh = C.c_void_p()
    assert lib.pa_batch_init(C.byref(cfg), 1, None, 0,
                             C.byref(bh)) == b.PA_EINVAL
    assert not bh.value
    cfg = b.pa_config()
    cfg.L, cfg.R_target, cfg.rng_mode = 8, 10, 2           # no such stream
    assert lib.pa_batch_init(C.byref(cfg), 1, None, 0,
                             C.byref(bh)) == b.PA_EINVAL
    assert not bh.value
    cfg = b.pa_config()                                    # Potts: words only
    cfg.L, cfg.R_target, cfg.model, cfg.q = 16, 10, b.PA_POTTS, 3
    cfg.rng_mode = b.PA_RNG_PLANES
    assert lib.pa_batch_init(C.byref(cfg), 1, None, 0,
                             C.byref(bh)) == b.PA_EINVAL
    assert not bh.value
    # Potts populations in a batch: the four-sites-per-word sizes, one byte
    # per state, 2 <= q <= 16
    for L, q, layout in ((12, 3, 0), (64, 1, 0), (64, 17, 0), (64, 3, 1)):
        cfg = b.pa_config()
        cfg.L, cfg.R_target, cfg.model, cfg.q = L, 10, b.PA_POTTS, q
        cfg.layout = layout
        assert lib.pa_batch_init(C.byref(cfg), 1, None, 0,
                                 C.byref(bh)) == b.PA_EINVAL, (L, q, layout)
        assert not bh.value
    assert lib.pa_sweep(None, 0.1, 1) == b.PA_EINVAL
    assert lib.pa_anneal(None, None, 0, 1, None, None, None) == b.PA_EINVAL
    assert lib.pa_resample(None, 0.1, None) == b.PA_EINVAL


def test_product_path_does_not_touch_the_oracle():
    """The package never imports, loads or names the oracle."""
    pkg = os.path.join(ROOT, "paper_2006_00561_amd")
    for dp, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dp, f)).read()
                assert "oracle" not in src.lower(), f


def _pop_file(path, L=4, R=2, spins=None, extra=b"", magic=b"PAPOPv04",
              fam=None, n0=None, R_hdr=None, cap_hdr=None, rng_mode=0,
              reserved=0):
    """A population file written from the documented layout: 112-byte
    header (its last words the founding population size, the sweep's
    random-number mode and a zero word), spins [R][L][L] int8, E and M
    int32, families uint32."""
    import struct
    N = L * L
    n0 = R if n0 is None else n0
    Rh = R if R_hdr is None else R_hdr
    cap = R + 100 if cap_hdr is None else cap_hdr
    hdr = magic + struct.pack("<qqqqdddiiiiIiiiiIii", R, cap, 1, Rh, 0.25,
                              N * 0.6931471805599453, 0.0, L, 0, 0, 1, 0, 3,
                              0, 0, 0, n0, rng_mode, reserved)
    assert len(hdr) == 112
    s = bytes([1] * (R * N)) if spins is None else spins
    E = struct.pack("<%di" % R, *([-2 * N] * R))
    M = struct.pack("<%di" % R, *([N] * R))
    F = struct.pack("<%dI" % R, *(range(R) if fam is None else fam))
    with open(path, "wb") as f:
        f.write(hdr + s + E + M + F + extra)


def test_load_rejects_bad_files_before_any_device_work(tmp_path):
    from paper_2006_00561_amd import binding as b
    lib = b.lib()
    h = C.c_void_p()
    missing = str(tmp_path / "missing.pa")
    assert lib.pa_load(missing.encode(), None, C.byref(h)) == b.PA_EIO
    bad = [("magic", dict(magic=b"NOTAPOP!")),
           ("older format", dict(magic=b"PAPOPv03")),
           ("random-number mode", dict(rng_mode=2)),
           ("reserved word", dict(reserved=1)),
           ("spin value", dict(spins=bytes([1] * 31 + [0]))),
           ("family number", dict(fam=[0, 2])),
           # a header that claims two billion replicas over a short body is
           # refused by its size, before anything is allocated
           ("size", dict(R_hdr=(1 << 31) - 1, cap_hdr=(1 << 32) - 1)),
           ("founding size", dict(n0=0)),
           ("trailing bytes", dict(extra=b"\x00"))]
    for name, kw in bad:
        p = str(tmp_path / (name.replace(" ", "_") + ".pa"))
        _pop_file(p, **kw)
        assert lib.pa_load(p.encode(), None, C.byref(h)) == b.PA_EIO, name
        assert not h.value
    p = str(tmp_path / "short.pa")
    _pop_file(p)
    with open(p, "r+b") as f:
        f.truncate(112 + 10)
    assert lib.pa_load(p.encode(), None, C.byref(h)) == b.PA_EIO
    assert lib.pa_save(None, p.encode()) == b.PA_EINVAL
    assert lib.pa_strerror(b.PA_EIO).decode().startswith("population file")


def test_product_path_fails_loudly_without_the_library():
    """Without libpa.so the binding raises: there is no CPU fallback, and no
    population can be made (run in a subprocess so that the loaded library
    of this process is untouched)."""
    import subprocess
    import sys
    code = ("import paper_2006_00561_amd.binding as b\n"
            "b.SO_PATH = '/nonexistent/libpa.so'\n"
            "b._lib = None\n"
            "try:\n"
            "    b.Population(8, 10)\n"
            "except RuntimeError as e:\n"
            "    print('raised:', e)\n"
            "else:\n"
            "    print('computed without the library')\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert "raised:" in r.stdout and "no fallback" in r.stdout, r.stdout
