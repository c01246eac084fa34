"""MI355X-native GOAT hot path: HIP kernels behind a C ABI (libgoat.so) and a
thin ctypes binding. Import the binding explicitly (``from
paper_2111_05366_amd import goat``); this package init loads nothing."""
