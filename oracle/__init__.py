"""FP64 CPU oracle for the mixture CAVI path.

Test infrastructure only: the tests, the smoke check and the benchmark's CPU
baseline leg use it; the GPU library never imports, links or calls it.
"""
