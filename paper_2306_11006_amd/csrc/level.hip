// level.hip -- one level ("wave", ArctyrEX Section 4.2) of a gate DAG.
//
// A level is evaluated by four launches on one stream, capturable into a
// HIP graph:
//   1. k_level_slots: one workgroup scans the gate list and gives every
//      bootstrapped gate its bootstrap slot(s) (MUX takes two), so the
//      bootstrap launch sees a dense batch; the slot count stays on the
//      device.
//   2. k_level_preop: the linear pre-op of every gate (Fig. 1 first box);
//      NOT / COPY / CONST write their output wire directly, bootstrapped
//      gates write their bootstrap input(s).
//   3. the bootstrap kernel of the chosen form over the dense slots;
//   4. the key switch, fused with the MUX combine, writing output wires.
// Gates with an unknown opcode or an out-of-range wire index get no slot
// and write nothing.
#include "internal.hpp"

namespace cggi {

int keyswitch_level(const Ctx *c, const cggi_gate_t *gates,
                    const int32_t *slot, const uint32_t *big,
                    uint32_t *wires, int G, int W, hipStream_t s);

namespace {

constexpr uint32_t MU = 1u << 29;

__device__ __forceinline__ bool in_range(int x, int W)
{
    return x >= 0 && x < W;
}

// number of inputs read by an opcode (-1: unknown)
__device__ __forceinline__ int op_inputs(int op)
{
    switch (op) {
    case CGGI_NAND: case CGGI_AND: case CGGI_OR: case CGGI_XOR:
    case CGGI_NOR: case CGGI_XNOR:
        return 2;
    case CGGI_MUX:
        return 3;
    case CGGI_NOT: case CGGI_COPY:
        return 1;
    case CGGI_CONST0: case CGGI_CONST1:
        return 0;
    default:
        return -1;
    }
}

__device__ __forceinline__ bool gate_valid(const cggi_gate_t &g, int W)
{
    int k = op_inputs(g.op);
    if (k < 0 || !in_range(g.out, W))
        return false;
    if (k >= 1 && !in_range(g.in0, W))
        return false;
    if (k >= 2 && !in_range(g.in1, W))
        return false;
    if (k >= 3 && !in_range(g.in2, W))
        return false;
    return true;
}

__device__ __forceinline__ int op_bootstraps(int op)
{
    switch (op) {
    case CGGI_MUX:
        return 2;
    case CGGI_NOT: case CGGI_COPY: case CGGI_CONST0: case CGGI_CONST1:
        return 0;
    default:
        return 1;
    }
}

constexpr int SLOT_THREADS = 1024;

__global__ __launch_bounds__(SLOT_THREADS) void k_level_slots(
    const cggi_gate_t *__restrict__ gates, int G, int W,
    int32_t *__restrict__ slot, int32_t *__restrict__ count)
{
    __shared__ int32_t part[SLOT_THREADS];
    const int tid = threadIdx.x;
    const int chunk = (G + SLOT_THREADS - 1) / SLOT_THREADS;
    const int lo = min(G, tid * chunk), hi = min(G, lo + chunk);
    int32_t mine = 0;
    for (int g = lo; g < hi; ++g) {
        cggi_gate_t gt = gates[g];
        if (gate_valid(gt, W))
            mine += op_bootstraps(gt.op);
    }
    part[tid] = mine;
    __syncthreads();
    // Hillis-Steele inclusive scan over the per-thread totals
    for (int off = 1; off < SLOT_THREADS; off <<= 1) {
        int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - mine;
    for (int g = lo; g < hi; ++g) {
        cggi_gate_t gt = gates[g];
        int k = gate_valid(gt, W) ? op_bootstraps(gt.op) : 0;
        slot[g] = k ? run : -1;
        run += k;
    }
    if (tid == SLOT_THREADS - 1)
        count[0] = part[tid];
}

__global__ __launch_bounds__(256) void k_level_preop(
    const cggi_gate_t *__restrict__ gates, const int32_t *__restrict__ slot,
    uint32_t *__restrict__ wires, uint32_t *__restrict__ small, int W, int n)
{
    const int g = blockIdx.x;
    const cggi_gate_t gt = gates[g];
    if (!gate_valid(gt, W))
        return;
    const size_t len = (size_t)n + 1;
    // inputs an opcode does not read may hold anything: point them at wire 0
    const uint32_t *x = wires + (size_t)(in_range(gt.in0, W) ? gt.in0 : 0) * len;
    const uint32_t *y = wires + (size_t)(in_range(gt.in1, W) ? gt.in1 : 0) * len;
    const uint32_t *z = wires + (size_t)(in_range(gt.in2, W) ? gt.in2 : 0) * len;
    uint32_t *o = wires + (size_t)gt.out * len;
    const int s = slot[g];
    uint32_t *b0 = s >= 0 ? small + (size_t)s * len : nullptr;
    for (int col = threadIdx.x; col <= n; col += blockDim.x) {
        const uint32_t cst = col == n ? 1u : 0u;   // trivial ciphertext (0,c)
        switch (gt.op) {
        case CGGI_NOT: o[col] = 0u - x[col]; break;
        case CGGI_COPY: o[col] = x[col]; break;
        case CGGI_CONST0: o[col] = cst * (0u - MU); break;
        case CGGI_CONST1: o[col] = cst * MU; break;
        case CGGI_NAND: b0[col] = cst * MU - x[col] - y[col]; break;
        case CGGI_AND: b0[col] = cst * (0u - MU) + x[col] + y[col]; break;
        case CGGI_OR: b0[col] = cst * MU + x[col] + y[col]; break;
        case CGGI_XOR: b0[col] = cst * (2u * MU) + 2u * (x[col] + y[col]); break;
        case CGGI_NOR: b0[col] = cst * (0u - MU) - x[col] - y[col]; break;
        case CGGI_XNOR:
            b0[col] = cst * (0u - 2u * MU) - 2u * (x[col] + y[col]);
            break;
        case CGGI_MUX:
            b0[col] = cst * (0u - MU) + x[col] + y[col];
            b0[len + col] = cst * (0u - MU) - x[col] + z[col];
            break;
        default: break;
        }
    }
}

} // namespace

int level_launch(Ctx *c, cggi_form_t form, const cggi_gate_t *gates, int G,
                 uint32_t *wires, int W, const LevelWs &ws, bool prof,
                 hipStream_t s)
{
    const Shape &sh = c->sh;
    Ctx *pc = prof ? c : nullptr;
    hipLaunchKernelGGL(k_level_slots, dim3(1), dim3(SLOT_THREADS), 0, s,
                       gates, G, W, ws.slot, ws.count);
    CGGI_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_level_preop, dim3(G), dim3(256), 0, s, gates,
                       ws.slot, wires, ws.small, W, sh.n);
    CGGI_HIP_TRY(hipGetLastError());
    int rc;
    {
        ProfScope ps(pc, 0, s);
        rc = form == CGGI_FORM_INT8
                 ? int8_bootstrap(c, ws.small, nullptr, ws.big, 2 * G,
                                  ws.count, s)
                 : ntt_bootstrap(c, ws.small, nullptr, ws.big, 2 * G,
                                 ws.count, s);
    }
    if (rc != CGGI_OK)
        return rc;
    ProfScope ps(pc, 1, s);
    return keyswitch_level(c, gates, ws.slot, ws.big, wires, G, W, s);
}

} // namespace cggi
