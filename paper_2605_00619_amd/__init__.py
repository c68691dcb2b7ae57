"""MI355X-native ADER-AFE-DG hot path: HIP kernels for gfx950 behind a C ABI
(include/afe.h), with a thin ctypes binding in `afe`."""
