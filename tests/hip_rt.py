"""The HIP runtime that the library itself runs on, reached through ctypes (test
plumbing only): device memory, free-memory queries and streams for the tests of
the library's options and of its entry point that allocates nothing.  It is looked
up by soname after the library is loaded, so the process keeps one runtime."""
import ctypes

_RT = None


def _rt():
    global _RT
    if _RT is None:
        import paper_2604_08374_amd as hb

        hb._lib()  # the library's own dependency is the runtime found below
        rt = ctypes.CDLL("libamdhip64.so.7")
        rt.hipMemGetInfo.argtypes = [ctypes.POINTER(ctypes.c_size_t)] * 2
        rt.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        rt.hipFree.argtypes = [ctypes.c_void_p]
        rt.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        rt.hipStreamDestroy.argtypes = [ctypes.c_void_p]
        for f in (rt.hipMemGetInfo, rt.hipMalloc, rt.hipFree, rt.hipStreamCreateWithFlags,
                  rt.hipStreamDestroy):
            f.restype = ctypes.c_int
        _RT = rt
    return _RT


def _ok(err, what):
    if err != 0:
        raise RuntimeError(f"{what} failed: HIP error {err}")


def mem_get_info():
    """(free, total) bytes of the current device."""
    free, total = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _ok(_rt().hipMemGetInfo(ctypes.byref(free), ctypes.byref(total)), "hipMemGetInfo")
    return free.value, total.value


def malloc(nbytes):
    p = ctypes.c_void_p(0)
    err = _rt().hipMalloc(ctypes.byref(p), nbytes)
    return p.value if err == 0 else 0


def free(ptr):
    _ok(_rt().hipFree(ctypes.c_void_p(ptr)), "hipFree")


def stream_create():
    s = ctypes.c_void_p(0)
    _ok(_rt().hipStreamCreateWithFlags(ctypes.byref(s), 1), "hipStreamCreateWithFlags")
    return s.value


def stream_destroy(s):
    _ok(_rt().hipStreamDestroy(ctypes.c_void_p(s)), "hipStreamDestroy")
