// Single translation unit of libpyst (device helpers are shared inline, and one
// unit keeps kernel launches and their definitions together).
#include "ctx.hip"
#include "ops.hip"
#include "agg.hip"
#include "query.hip"
#include "fast.hip"
#include "pack.hip"
#include "stream.hip"
#include "batch.hip"
#include "server.hip"
