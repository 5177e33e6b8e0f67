"""The largest lattices the C ABI accepts, per velocity set and storage: each
population buffer stays below 4 GiB (Q x (nx ny + 3840) x bytes < 2^32, the
reach of the kernels' 32-bit buffer offsets); one more row is rejected."""

# name: (velocity set, storage, nx, ny)
MAX_LATTICES = {
    "q9_f32": (9, "f32", 16384, 7281),
    "q9_f16dev": (9, "f16dev", 16384, 14563),
    "q9_f64": (9, "f64", 8192, 7281),
    "q21_f32": (21, "f32", 8192, 6241),
    "q21_f64": (21, "f64", 8192, 3120),
}

STORAGE_BYTES = {"f32": 4, "f16dev": 2, "f64": 8}


def buffer_bytes(q, storage, nx, ny):
    """The bound the C ABI checks: Q x (nx ny + 3840) x bytes per element."""
    return q * (nx * ny + 3840) * STORAGE_BYTES[storage]
