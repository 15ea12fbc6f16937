"""MI355X (gfx950) group tree-walk gravity: host FP64 octree, HIP walk and
FP32 compensated evaluation behind the C ABI of include/octgrav.h."""
