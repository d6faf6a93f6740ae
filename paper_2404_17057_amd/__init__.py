"""MI355X-native hot path of the compressible-gas Material Point Method of
arXiv 2404.17057: a C-ABI library of gfx950 HIP kernels (libmpm.so) and a
thin ctypes binding.  Importing the package loads nothing; the binding loads
the library on first use and fails loudly if it is missing."""
