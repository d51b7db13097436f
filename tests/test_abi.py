"""The C-ABI library loads without a GPU and exports every entry point of include/reco.h;
the Python binding declares exactly those functions."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "reco.h")
LIB = os.path.join(ROOT, "paper_1310_0956_amd", "libreco.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(reco_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_expected_entry_points():
    names = declared()
    for must in ("reco_create_geometry", "reco_project", "reco_backproject", "reco_wmg_apply",
                 "reco_solve_cgls", "reco_solve_gmres", "reco_solve_sirt", "reco_solve_batch",
                 "reco_submit", "reco_poll", "reco_server_create", "reco_server_destroy",
                 "reco_destroy_geometry", "reco_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "libreco.so not built"
    lib = ctypes.CDLL(LIB)
    missing = [s for s in declared() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_header():
    import paper_1310_0956_amd as reco
    assert sorted(reco.EXPORTED) == declared()


def test_invalid_arguments_rejected_without_gpu_work():
    import paper_1310_0956_amd as reco
    lib = reco._lib
    out = ctypes.c_void_p()
    bad = [reco.GeometryDesc(0, 10, 10, 2, 0, 0), reco.GeometryDesc(16, 0, 10, 2, 0, 0),
           reco.GeometryDesc(16, 10, 10, 7, 0, 0), reco.GeometryDesc(18, 10, 10, 3, 0, 0),
           reco.GeometryDesc(16, 10, 10, 2, 5, 0), reco.GeometryDesc(16, 10, 10, 2, 0, 2),
           # 32-bit byte offsets: padded image (n + 32) (n + 8) and sinogram below 2^31 bytes
           reco.GeometryDesc(23151, 1, 1, 1, 0, 0), reco.GeometryDesc(16365, 1, 1, 1, 1, 0),
           reco.GeometryDesc(64, 1 << 15, 1 << 14, 1, 0, 0),
           reco.GeometryDesc(64, 1 << 14, 1 << 14, 1, 1, 0)]
    for d in bad:
        rc = lib.reco_create_geometry(ctypes.byref(d), None, ctypes.byref(out))
        assert rc == reco.RECO_EINVAL, (d.n, d.n_angles, rc)
        assert reco.last_error()
    assert lib.reco_create_geometry(None, None, ctypes.byref(out)) == reco.RECO_EINVAL
    assert lib.reco_project(None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_solve_cgls(None, None, None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_solve_cgls_noalloc(None, None, None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_solve_batch(-1, None, None, None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_solve_batch(0, None, None, None, None, None, None) == reco.RECO_OK
    assert lib.reco_solve_batch(1, None, None, None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_server_create(0, 4, ctypes.byref(out)) == reco.RECO_EINVAL
    assert lib.reco_server_create(1 << 20, 0, ctypes.byref(out)) == reco.RECO_EINVAL
    assert lib.reco_server_create(1 << 20, 4, None) == reco.RECO_EINVAL
    assert lib.reco_submit(None, None, None, None, None, None) == reco.RECO_EINVAL
    assert lib.reco_poll(None, 1, None, None) == reco.RECO_EINVAL
    assert lib.reco_server_destroy(None) == reco.RECO_OK


_CTYPE = {"int32_t": ctypes.c_int32, "reco_status": ctypes.c_int32, "double": ctypes.c_double,
          "double*": ctypes.POINTER(ctypes.c_double)}


def _header_struct(name):
    """(field, C type) pairs of `typedef struct { ... } name;` in the header."""
    txt = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*" + name + r"\s*;", txt).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        m = re.match(r"(\w+)\s*(\*?)\s*(\w+)$", decl)
        fields.append((m.group(3), m.group(1) + m.group(2)))
    return fields


def test_binding_structs_match_header():
    """The ctypes structures have the header's fields, in order, with the same types
    (so sizes and offsets agree)."""
    import paper_1310_0956_amd as reco
    for cname, py in (("reco_geometry_desc", reco.GeometryDesc), ("reco_solve_opts", reco.SolveOpts),
                      ("reco_solve_info", reco.SolveInfo)):
        hdr = _header_struct(cname)
        assert len(hdr) == len(py._fields_), cname
        for (hname, htype), (_, ptype) in zip(hdr, py._fields_):
            want = _CTYPE[htype]
            assert ctypes.sizeof(ptype) == ctypes.sizeof(want), (cname, hname)
            assert type(ptype) is type(want) or ptype is want, (cname, hname)
    assert [f for f, _ in _header_struct("reco_geometry_desc")][-1] == "projector"
    assert reco.PROJ_EXACT == 0 and reco.PROJ_JOSEPH == 1


def test_noalloc_scratch_size_matches_header():
    import paper_1310_0956_amd as reco
    txt = open(HEADER).read()
    m = re.search(r"#define RECO_NOALLOC_SCRATCH_BYTES \((\d+)u \* 1024u \* 1024u\)", txt)
    assert m and int(m.group(1)) * 1024 * 1024 == reco.NOALLOC_SCRATCH_BYTES
