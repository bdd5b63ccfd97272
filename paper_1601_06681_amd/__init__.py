"""MI355X-native eHDG iteration: HIP kernels behind a C ABI (libehdg.so), with a thin
ctypes binding.  Importing the package does not load the library; the first call
into `paper_1601_06681_amd.ehdg` does, and raises if it has not been built."""
