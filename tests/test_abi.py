"""The C ABI: libpe.so loads without a GPU and exports every entry point that
include/pe.h declares (no compute call is made here)."""
import ctypes
import os
import re
import subprocess

from paper_2410_05190_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "pe.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pe_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("pe_metric", "pe_draw", "pe_loglike_batch", "pe_weights_ess", "pe_event_create",
                 "pe_event_destroy", "pe_last_error"):
        assert must in names
    assert set(names) == set(binding.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name


def test_binding_declares_every_signature():
    L = binding.load()
    for name in binding.EXPORTS:
        f = getattr(L, name)
        assert f.argtypes is not None, name
        assert f.restype is not None, name


def test_binding_loads_and_pure_host_calls():
    L = binding.load()
    assert binding.pe_dim(binding.PE_PARAMS_4D) == 4
    assert binding.pe_dim(binding.PE_PARAMS_11D) == 11
    assert binding.pe_dim(7) == 0
    # argument errors are caught on the host before any device work
    d = binding.make_desc(0, 10, 20.0, 0.25)
    h = ctypes.c_void_p()
    st = L.pe_event_create(ctypes.byref(d), None, None, None, ctypes.byref(h))
    assert st == 1 and h.value is None
    assert "n_det" in binding.pe_last_error()
    assert L.pe_set_chunks(65) == 1
    assert L.pe_set_chunks(-1) == 1
    assert L.pe_set_chunks(0) == 0
    assert L.pe_set_plan(100, 1024) == 1 and L.pe_set_plan(16384, 16) == 1
    assert binding.pe_get_plan() == (16384, 1024)
    assert L.pe_autotune_plan(0, None, None, None, 1, 0, None, None, None, None) == 1
    assert L.pe_loglike_batch(None, None, 0, 0, None, None, None) == 1
    # an empty multi-event batch is a no-op; bad arrays are rejected on the host
    assert L.pe_loglike_multi(0, None, None, None, 1, None, None, None) == 0
    assert L.pe_loglike_multi(2, None, None, None, 1, None, None, None) == 1
    assert L.pe_loglike_multi(0, None, None, None, 7, None, None, None) == 1


def test_proposal_update_and_refine_argument_errors_on_host():
    L = binding.load()
    assert L.pe_proposal_update(None, None, None, 0, None, None, None, None) == 1
    assert "event is NULL" in binding.pe_last_error()
    assert L.pe_refine(None, None, None, 1, 16, 0, 1, None, None, None, None, None, None, None) == 1


def test_tile_entry_points_reject_bad_arguments_on_host():
    L = binding.load()
    sl = binding.make_slice([1.0] * 4, [[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, 0], [0, 0, 0, 1.0]], 2.0)
    # pe_slice_t: 11 + 121 + 1 doubles, uint32 sub_mask, padded to 8 bytes
    assert ctypes.sizeof(binding.Slice) == (11 + 121 + 1) * 8 + 8
    assert binding.Slice.sub_mask.offset == (11 + 121 + 1) * 8
    assert L.pe_slice_sample(None, ctypes.byref(sl), 0, 0, 0, 10, None, None, None, None, None) == 1
    assert L.pe_tile_bank(None, ctypes.byref(sl), 1.0, 0, 0, 16, 16, 0.1, 4, None, None, None, None, None) == 1
    assert L.pe_tile_assign(5, 1, None, 1, 0, None, 0, None, None) == 1
    assert "dim" in binding.pe_last_error()
    assert L.pe_tile_assign(4, 0, None, 1, 0, None, 0, None, None) == 1
    assert L.pe_tile_draw(1, None, 1, None, None, 4, None, 1, 0, 0, 1, None, None, None, None, None) == 1
    assert L.pe_tile_extrinsic(None, None, None, 0xF, 0, 0, 0, 1, None, None, None, None) == 1
    assert "event is NULL" in binding.pe_last_error()


def test_batch_item_layout_matches_header():
    # pe_batch_item_t: 5 pointers, int32, uint32, uint64, pointer, int64, 7 pointers
    assert ctypes.sizeof(binding.BatchItem) == 5 * 8 + 4 + 4 + 8 + 8 + 8 + 7 * 8


def test_batch_run_argument_errors_on_host():
    L = binding.load()
    assert L.pe_batch_run(0, None, binding.PE_STAGE_ALL, 1, None) == 0
    assert L.pe_batch_run(1, None, binding.PE_STAGE_ALL, 1, None) == 1
    assert L.pe_batch_run(0, None, 64, 1, None) == 1
    it = binding.BatchItem()
    arr = (binding.BatchItem * 1)(it)
    assert L.pe_batch_run(1, ctypes.cast(arr, ctypes.c_void_p), binding.PE_STAGE_LOGLIKE, 1, None) == 1
    assert "event is NULL" in binding.pe_last_error()


def test_mixture_logq_argument_errors_on_host():
    L = binding.load()
    w = (ctypes.c_double * 2)(1.0, 1.0)
    assert L.pe_mixture_logq(None, 2, ctypes.cast(w, ctypes.c_void_p), None, None, None, 0, None, None) == 1
    assert "event is NULL" in binding.pe_last_error()
    assert binding.PE_MIX_MAX == 16


def test_server_structs_and_host_checks():
    # pe_server_config_t: int64, 2 int32, double, 4 int32
    assert ctypes.sizeof(binding.ServerConfig) == 8 + 8 + 8 + 16
    # pe_request_t: desc, 2 pointers, 2 int32, pointer, uint64, uint32, int32, int64, 3 pointers
    assert ctypes.sizeof(binding.Request) == ctypes.sizeof(binding.EventDesc) + 16 + 8 + 8 + 8 + 8 + 8 + 24
    # pe_result_t: int64, 2 int32, 4 double, 3 double
    assert ctypes.sizeof(binding.Result) == 8 + 8 + 32 + 24
    L = binding.load()
    h = ctypes.c_void_p()
    bad = binding.ServerConfig(1 << 10, 1, 16, 8.0, 1, 0, 0, 0)  # budget below 1 MiB
    assert L.pe_server_create(ctypes.byref(bad), ctypes.byref(h)) == 1 and h.value is None
    bad = binding.ServerConfig(1 << 30, 1, 0, 8.0, 1, 0, 0, 0)  # no slots
    assert L.pe_server_create(ctypes.byref(bad), ctypes.byref(h)) == 1
    bad = binding.ServerConfig(1 << 30, 1, 16, 0.0, 1, 0, 0, 0)  # no slice time
    assert L.pe_server_create(ctypes.byref(bad), ctypes.byref(h)) == 1
    bad = binding.ServerConfig(1 << 30, 1, 16, 8.0, 1, 0, 100, 0)  # plan out of range
    assert L.pe_server_create(ctypes.byref(bad), ctypes.byref(h)) == 1
    assert L.pe_server_destroy(None) == 1
    assert L.pe_server_tune(None, 1, None, None, None, 1) == 1
    assert L.pe_server_busy(None, None) == 1
    c = ctypes.c_int32()
    assert L.pe_server_plans(None, 0, None, None, ctypes.byref(c)) == 1


def test_event_desc_layout_matches_header(tmp_path):
    """The binding's pe_event_desc_t has the header's size and field offsets, as the C compiler
    lays the header's struct out."""
    fields = [f[0] for f in binding.EventDesc._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "pe.h"\nint main(void) {\n'
                   '    printf("%zu\\n", sizeof(pe_event_desc_t));\n' +
                   "".join(f'    printf("%zu\\n", offsetof(pe_event_desc_t, {f}));\n' for f in fields) +
                   "    return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    vals = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert vals[0] == ctypes.sizeof(binding.EventDesc)
    assert vals[1:] == [getattr(binding.EventDesc, f).offset for f in fields]
