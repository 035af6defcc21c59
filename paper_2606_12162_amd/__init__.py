"""MI355X-native explicit time step of the hyperbolic Serre-Green-Naghdi
system coupled to the shallow water equations (HIP kernels behind the C ABI
in include/hsgn.h; this package holds the kernels' sources, their build and a
thin ctypes binding)."""
