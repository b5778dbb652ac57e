// dvc_lib.hip -- the library's single translation unit.  Device globals
// (error word, work queues) are defined once in dvc_internal.hpp and shared
// by every kernel without relocatable device code.
#include "rollout.hip"
#include "gen.hip"
#include "valuenet.hip"
#include "search.hip"
#include "capi.hip"
