"""MI355X-native HDR-fused ptychography: MNF exposure fusion and mini-batched
ePIE/rPIE reconstruction, hand-written HIP kernels behind a C ABI."""
