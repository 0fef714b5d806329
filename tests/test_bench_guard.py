"""bench.py starts no worker process under a profiler: with a rocprofiler
tool preloaded every child process would initialise the GPU under it."""
import multiprocessing

import bench


def test_profiler_detection():
    assert bench.profiler_active({"LD_PRELOAD": "/opt/rocm/lib/rocprofiler-sdk/librocprofiler-sdk-tool.so"})
    assert bench.profiler_active({"ROCPROF_KERNEL_TRACE": "1"})
    assert bench.profiler_active({"ROCP_TOOL_LIBRARIES": "x"})
    assert not bench.profiler_active({"LD_PRELOAD": "", "PATH": "/usr/bin"})


def test_cpu_baseline_starts_no_pool_under_profiler(monkeypatch):
    monkeypatch.setenv("ROCPROF_KERNEL_TRACE", "1")

    def no_pool(*a, **k):
        raise AssertionError("a process pool was started under a profiler")

    monkeypatch.setattr(multiprocessing, "get_context", no_pool)
    monkeypatch.setattr(multiprocessing, "Pool", no_pool)
    assert bench.cpu_baseline([None], None, None, 4) is None
