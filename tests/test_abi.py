"""The C-ABI library loads and exports every entry point of include/gd.h, and
rejects bad arguments on the host before anything is enqueued (no GPU needed)."""
import ctypes as C
import math
import os
import re

import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_2609_35967_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2609_35967_amd import build
        build.build()
    return binding.load()


def _declared():
    src = open(os.path.join(ROOT, "include", "gd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(gd_[a-z_]+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert {"gd_build_neighbors", "gd_collision_rates", "gd_sample_collisions", "gd_push"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name
    from paper_2609_35967_amd import binding
    assert set(binding.EXPORTS) == set(names)
    assert lib.gd_version().startswith(b"gd ")


def test_struct_layout_matches_header(tmp_path):
    from paper_2609_35967_amd import binding
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include "gd.h"\nint main(){printf("%zu %zu %zu %zu", sizeof(gd_problem),'
                   ' sizeof(gd_particles), sizeof(gd_interval), sizeof(gd_neighbors));}\n')
    import subprocess
    exe = tmp_path / "sz"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    want = [C.sizeof(binding.GdProblem), C.sizeof(binding.GdParticles), C.sizeof(binding.GdInterval),
            C.sizeof(binding.GdNeighbors)]
    assert got == want


def test_host_validation(lib):
    from paper_2609_35967_amd import binding
    P = binding.make_problem(workloads.disk3d_params(1000))
    sz = C.c_size_t()
    assert lib.gd_workspace_size(C.byref(P), C.byref(sz)) == 0 and sz.value > 0
    bad = binding.make_problem(dict(workloads.disk3d_params(1000), k=257))
    assert lib.gd_workspace_size(C.byref(bad), C.byref(sz)) == -1
    assert b"k = 257" in lib.gd_last_error()
    ok = binding.make_problem(dict(workloads.disk3d_params(1000), k=256))
    assert lib.gd_workspace_size(C.byref(ok), C.byref(sz)) == 0
    bad = binding.make_problem(dict(workloads.const_box_params(1000), t0=0.0))
    assert lib.gd_workspace_size(C.byref(bad), C.byref(sz)) == -1
    assert lib.gd_interval_init(None, 1.0, None) == -1
    s = binding.GdParticles()
    nb = binding.GdNeighbors()
    # NULL arrays are rejected before any launch
    assert lib.gd_build_neighbors(C.byref(P), C.byref(s), C.byref(s), C.byref(nb), None, 0, None) == -1
    assert lib.gd_push(C.byref(P), None, None, 1.0, None, 0, None) == -1
    assert lib.gd_status_read(None, None, None) == -1
    # a workspace that is too small is reported as such
    fake = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M", "r", "th", "ph", "vr", "lth", "lph"):
        setattr(fake, k, 256)
    fake.m[0] = 256
    fake.m[1] = 512
    other = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M", "r", "th", "ph", "vr", "lth", "lph"):
        setattr(other, k, 1024)
    other.m[0] = 1024
    other.m[1] = 2048
    nb = binding.GdNeighbors(4096, 4096, 4096, None)
    rc = lib.gd_build_neighbors(C.byref(P), C.byref(fake), C.byref(other), C.byref(nb), C.c_void_p(256), 16, None)
    assert rc == -2 and b"workspace" in lib.gd_last_error()
    rc = lib.gd_build_neighbors(C.byref(P), C.byref(fake), C.byref(fake), C.byref(nb), C.c_void_p(256), 1 << 40, None)
    assert rc == -1 and b"alias" in lib.gd_last_error()
    rc = lib.gd_sample_collisions(C.byref(P), C.byref(fake), C.byref(nb), C.c_void_p(256), C.c_void_p(256), 1,
                                  1 << 33, None, None, 0, C.c_void_p(256), 1 << 40, None)
    assert rc == -1 and b"interval_index" in lib.gd_last_error()


def test_sample_table_validation(lib):
    # the calls that share the deferred sampling pass between runs reject bad
    # tables, slots and arguments before any launch
    from paper_2609_35967_amd import binding
    P = binding.make_problem(workloads.local_box_params(1000))
    sz = C.c_size_t()
    assert lib.gd_sample_table_size(0, C.byref(sz)) == -1
    assert lib.gd_sample_table_size(4097, C.byref(sz)) == -1
    assert lib.gd_sample_table_size(1, None) == -1
    assert lib.gd_sample_table_size(8, C.byref(sz)) == 0
    one = C.c_size_t()
    assert lib.gd_sample_table_size(1, C.byref(one)) == 0
    assert sz.value > one.value > 0
    # a table run that does not fit its table, or with bad k / rates form
    assert lib.gd_sample_table_run(None, sz.value, 8, 32, 0, None) == -1
    assert lib.gd_sample_table_run(C.c_void_p(256), one.value, 8, 32, 0, None) == -1
    assert lib.gd_sample_table_run(C.c_void_p(256), sz.value, 8, 257, 0, None) == -1
    assert lib.gd_sample_table_run(C.c_void_p(256), sz.value, 8, 32, 2, None) == -1
    fake = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M", "r", "th", "ph", "vr", "lth", "lph"):
        setattr(fake, k, 256)
    fake.m[0] = 256
    fake.m[1] = 512
    nb = binding.GdNeighbors(4096, 4096, 4096, None)
    args = (C.byref(P), C.byref(fake), C.byref(nb), C.c_void_p(256), C.c_void_p(256), 1, 0, None, None, 0,
            C.c_void_p(256), 1 << 40)
    assert lib.gd_sample_collisions_deferred(*args, None, sz.value, 0, None) == -1
    assert b"table" in lib.gd_last_error()
    assert lib.gd_sample_collisions_deferred(*args, C.c_void_p(4096), sz.value, 8, None) == -1
    assert b"slot" in lib.gd_last_error()
    assert lib.gd_sample_collisions_deferred(*args, C.c_void_p(4096), sz.value, -1, None) == -1
    assert lib.gd_sample_audit(C.byref(P), C.byref(fake), None, C.c_void_p(256), 1 << 40, None) == -1


def test_problem_rmax_default_is_infinite():
    from paper_2609_35967_amd import binding
    assert math.isinf(binding.make_problem(workloads.const_box_params()).rmax)


def test_diffuse_validation(lib):
    # gd_diffuse checks its form, arrays, Schmidt numbers and step on the host
    from paper_2609_35967_amd import binding
    base = workloads.diffusion_ring_params("concentration", n=1000, axisym=0)
    full = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M", "r", "th", "ph", "vr", "lth", "lph"):
        setattr(full, k, 256)
    full.m[0] = 256
    P = binding.make_problem(base)
    assert lib.gd_diffuse(C.byref(P), None, 1.0, 1, 0, None) == -1
    part = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M"):
        setattr(part, k, 256)
    assert lib.gd_diffuse(C.byref(P), C.byref(part), 1.0, 1, 0, None) == -1
    assert b"lph" in lib.gd_last_error()
    assert lib.gd_diffuse(C.byref(P), C.byref(full), -1.0, 1, 0, None) == -1
    assert lib.gd_diffuse(C.byref(P), C.byref(full), math.inf, 1, 0, None) == -1
    bad = binding.make_problem(dict(base, Sc=(1.0, 1.0, 0.0)))
    assert lib.gd_diffuse(C.byref(bad), C.byref(full), 1.0, 1, 0, None) == -1
    assert b"Schmidt" in lib.gd_last_error()
    # the vertical Schmidt number is not used by a vertically integrated disk
    ok = binding.make_problem(dict(base, Sc=(1.0, 0.0, 1.0)))
    zero = binding.make_problem(dict(base, Sc=(1.0, 0.0, 1.0)), n=0)
    assert lib.gd_diffuse(C.byref(zero), C.byref(full), 1.0, 1, 0, None) == 0
    bad = binding.make_problem(dict(base, St_diff=-1.0))
    assert lib.gd_diffuse(C.byref(bad), C.byref(full), 1.0, 1, 0, None) == -1
    bad = binding.make_problem(dict(base, St_diff=0.0))
    nom = binding.GdParticles.from_buffer_copy(full)
    nom.m[0] = None
    assert lib.gd_diffuse(C.byref(bad), C.byref(nom), 1.0, 1, 0, None) == -1
    assert b"m[cur]" in lib.gd_last_error()
    bad = binding.make_problem(base)
    bad.diffusion = 3
    assert lib.gd_diffuse(C.byref(bad), C.byref(full), 1.0, 1, 0, None) == -1
    # no diffusion: nothing to check, nothing enqueued
    off = binding.make_problem(dict(base, diffusion="none"))
    assert lib.gd_diffuse(C.byref(off), None, -1.0, 1, 0, None) == 0
    assert ok.vint == 1


def test_group_call_validation(lib):
    # the spatial-group calls reject bad group tables, ranges and interval limits
    from paper_2609_35967_amd import binding
    P = binding.make_problem(workloads.const_box_params(1000))
    nb = binding.GdNeighbors(4096, 4096, 4096, None)
    fake = binding.GdParticles()
    for k in ("id", "x", "y", "z", "M"):
        setattr(fake, k, 256)
    fake.m[0] = 256
    fake.m[1] = 512
    lo = (C.c_int32 * 3)(0, 500, 1000)
    assert lib.gd_group_interactions(C.byref(P), C.byref(nb), lo, 0, C.c_void_p(256), None) == -1
    assert lib.gd_group_interactions(C.byref(P), C.byref(nb), lo, 65, C.c_void_p(256), None) == -1
    assert lib.gd_group_interactions(C.byref(P), C.byref(nb), lo, 2, None, None) == -1
    bad = (C.c_int32 * 3)(0, 500, 500)
    assert lib.gd_group_interactions(C.byref(P), C.byref(nb), bad, 2, C.c_void_p(256), None) == -1
    assert b"non-empty" in lib.gd_last_error()
    over = (C.c_int32 * 3)(0, 500, 1001)
    assert lib.gd_group_interactions(C.byref(P), C.byref(nb), over, 2, C.c_void_p(256), None) == -1
    ws = (C.c_void_p(256), 1 << 40)
    args = (C.byref(P), C.byref(fake), C.byref(nb), C.c_void_p(256), C.c_void_p(256))
    dev = (C.c_void_p(512), C.c_void_p(768))
    assert lib.gd_collision_rates_group(*args, 10, 5, 0, 2, *dev, 1, *ws, None) == -1
    assert b"range" in lib.gd_last_error()
    assert lib.gd_collision_rates_group(*args, 0, 1001, 0, 2, *dev, 1, *ws, None) == -1
    assert lib.gd_collision_rates_group(*args, 0, 10, 2, 2, *dev, 1, *ws, None) == -1
    assert lib.gd_collision_rates_group(*args, 0, 10, 0, 65, *dev, 1, *ws, None) == -1
    assert lib.gd_collision_rates_group(*args, 0, 10, 0, 2, None, dev[1], 1, *ws, None) == -1
    assert b"sched" in lib.gd_last_error()
    assert lib.gd_sample_collisions_group(*args, 1, 1 << 32, 0, 10, None, *ws, None) == -1
    assert lib.gd_sample_collisions_group(*args, 1, 0, -1, 10, None, *ws, None) == -1
    assert lib.gd_publish_group(C.byref(P), C.byref(fake), 5, 1001, None, 0, None) == -1
    assert lib.gd_publish_group(C.byref(P), C.byref(fake), 0, 10, C.c_void_p(512), 64, None) == -1


def test_static_reshuffle_rejects_sizes_beyond_its_table(lib):
    # the allocation-free entry point keeps pi's table in a fixed per-GPU array
    # of GD_RESHUFFLE_STATIC_MAX entries; a larger n fails on the host, before
    # any device work, with a message that names the limit
    from paper_2609_35967_amd import binding
    limit = 1 << 22
    src = open(os.path.join(ROOT, "include", "gd.h")).read()
    assert "#define GD_RESHUFFLE_STATIC_MAX (1 << 22)" in src
    nb = binding.GdNeighbors(256, 512, 768, 1024)  # never dereferenced: validation fails first
    P = binding.make_problem(workloads.const_box_params(limit + 1))
    assert lib.gd_reshuffle_neighbors_static(C.byref(P), C.byref(nb), 1, 0, None) == -1
    assert b"exceeds its fixed table of 4194304 entries" in lib.gd_last_error()
    assert lib.gd_reshuffle_neighbors_static(C.byref(P), None, 1, 0, None) == -1


def test_many_and_stream_validation(lib):
    from paper_2609_35967_amd.binding import GdManyTuning, GdRun
    out = C.c_void_p(123)
    runs = (GdRun * 1)()
    assert lib.gd_many_create(runs, 0, None, C.byref(out)) == -1 and not out.value
    assert b"nrun" in lib.gd_last_error()
    assert lib.gd_many_create(runs, 4097, None, C.byref(out)) == -1
    assert lib.gd_many_create(runs, 1, None, None) == -1
    bad = GdManyTuning(knn_tile=2)
    assert lib.gd_many_create(runs, 1, C.byref(bad), C.byref(out)) == -1
    assert b"tuning" in lib.gd_last_error()
    # a run with no problem is rejected, named by its index
    assert lib.gd_many_create(runs, 1, None, C.byref(out)) == -1
    assert b"run 0" in lib.gd_last_error()
    assert lib.gd_many_interval(None, None) == -1
    assert lib.gd_many_destroy(None) == 0
    par = C.c_int32()
    assert lib.gd_many_parity(None, C.byref(par)) == -1
    st = C.c_void_p(5)
    mask = (C.c_uint32 * 8)()
    assert lib.gd_stream_create_cu_mask(mask, 8, C.byref(st)) == -1 and not st.value
    assert b"no CU" in lib.gd_last_error()
    assert lib.gd_stream_create_cu_mask(None, 8, C.byref(st)) == -1
    assert lib.gd_stream_destroy(None) == 0


def test_transport_dt_validation(lib):
    from paper_2609_35967_amd.binding import GdNeighbors, GdParticles, GdStepLimits, make_problem
    P = make_problem(workloads.disk3d_params(1024))
    s = GdParticles()
    nb = GdNeighbors()
    lim = GdStepLimits(1.0, math.inf, 0.05, 0.5, 0.5)
    dt = C.c_void_p(64)
    assert lib.gd_transport_dt(C.byref(P), None, C.byref(nb), C.byref(lim), None, dt, None, 0, None) == -1
    assert lib.gd_transport_dt(None, C.byref(s), C.byref(nb), C.byref(lim), None, dt, None, 0, None) == -1
