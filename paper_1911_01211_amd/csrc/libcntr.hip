// Single translation unit of the HIP library (constant-memory weight tables
// are shared by every kernel without relocatable device code).
#include "weights.cpp"
#include "step.hip"
#include "vie2.hip"
#include "misc.hip"
#include "mats.hip"
#include "adjoint.hip"
#include "free.hip"
#include "kspace.hip"
#include "holstein.hip"
#include "api.cpp"
