"""MI355X-native multilayer-graph Laplacian engine: Gaussian-kernel W and
L_sym matvecs (NFFT fast summation and direct tiles), FP64 block Lanczos, and
the Allen--Cahn classifier, behind the C ABI of include/mlg.h."""
