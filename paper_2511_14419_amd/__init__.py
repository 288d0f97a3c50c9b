"""MI355X-native FlowRoI hot path: dense two-frame flow -> RoI mask.

The compute lives in ``libflowroi.so`` (HIP kernels for gfx950 behind a C
ABI declared in ``include/flowroi.h``). ``paper_2511_14419_amd.flowroi``
binds it; importing this package does not load the library.
"""
