// fk_chain.cpp -- chain rewriting done once per plan (no HIP).
#include "fk_chain.hpp"

#include <cstdint>
#include <cstring>
#include <utility>

// --------------------------------------------------------- normalisation --

// Run-time op list: swaps moved to the read (each later-crossed op's
// per-channel constants permuted), CVT dropped, SUB -> ADD(-k), and unless
// strict, MUL immediately followed by ADD -> FMA.  Every rewrite preserves
// the per-element fp32 arithmetic exactly except the contraction.  A loop
// becomes a LOOP record after its body's records; contraction pairs only
// records of one run: a loop body, or the stretch between two loop
// boundaries (a MUL that repeats cannot absorb an ADD that does not).
// Finally, runs of identical records become one record and a LOOP.
void fk::normalise_chain(const fk_chain_desc *ch, bool strict, std::vector<OpRec> &ops,
                         int32_t &swap)
{
    const int C = ch->read.channels;
    // swaps after op i (parity)
    std::vector<int> after(ch->n_ops + 1, 0);
    for (int i = ch->n_ops - 1; i >= 0; --i)
        after[i] = after[i + 1] ^ (ch->ops[i].kind == FK_OP_SWAP_RB ? 1 : 0);
    swap = (C >= 3) ? after[0] : 0;
    std::vector<OpRec> lin;
    std::vector<int> run;  // run id of each record in `lin`
    int cur = 0;
    for (int i = 0; i < ch->n_ops; ++i) {
        const fk_op_desc &d = ch->ops[i];
        if (d.kind == FK_OP_SWAP_RB || d.kind == FK_OP_CVT_F32)
            continue;
        OpRec r;
        std::memset(&r, 0, sizeof r);
        if (d.kind == FK_OP_LOOP) {
            // the body's ops are arithmetic, one record each: the last loop_span
            const int body = ++cur;
            for (size_t j = lin.size() - (size_t)d.loop_span; j < lin.size(); ++j)
                run[j] = body;
            r.code = OPC_LOOP;
            r.count = d.loop_count;
            lin.push_back(r);
            run.push_back(++cur);
            ++cur;
            continue;
        }
        float k[4];
        for (int c = 0; c < 4; ++c)
            k[c] = d.n_consts == 1 ? d.consts[0] : (c < C ? d.consts[c] : 0.0f);
        if (C >= 3 && after[i + 1] && d.n_consts != 1)
            std::swap(k[0], k[2]);
        switch (d.kind) {
        case FK_OP_MUL: r.code = OPC_MUL; break;
        case FK_OP_ADD: r.code = OPC_ADD; break;
        case FK_OP_SUB:
            r.code = OPC_ADD;
            for (int c = 0; c < 4; ++c)
                k[c] = -k[c];
            break;
        default: r.code = OPC_DIV; break;
        }
        for (int c = 0; c < 4; ++c)
            r.a[c] = k[c];
        lin.push_back(r);
        run.push_back(cur);
    }
    ops.clear();
    std::vector<int> orun;
    for (size_t i = 0; i < lin.size(); ++i) {
        if (!strict && lin[i].code == OPC_MUL && i + 1 < lin.size() &&
            lin[i + 1].code == OPC_ADD && run[i] == run[i + 1]) {
            OpRec f = lin[i];
            f.code = OPC_FMA;
            for (int c = 0; c < 4; ++c)
                f.b[c] = lin[i + 1].a[c];
            ops.push_back(f);
            ++i;
        } else {
            ops.push_back(lin[i]);
        }
        orun.push_back(run[i]);
    }
    // a LOOP's span: the records of its body, the run just before it
    for (size_t k = 0; k < ops.size(); ++k) {
        if (ops[k].code != OPC_LOOP)
            continue;
        int n = 0;
        for (size_t j = k; j > 0 && orun[j - 1] == orun[k - 1]; --j)
            ++n;
        ops[k].span = n;
    }
    merge_repeats(ops);
}

static bool same_record(const fk::OpRec &x, const fk::OpRec &y)
{
    return x.code == y.code && std::memcmp(x.a, y.a, sizeof x.a) == 0 &&
           std::memcmp(x.b, y.b, sizeof x.b) == 0;
}

// Consecutive identical records outside multi-record loop bodies, each
// possibly repeated by a one-record LOOP, become one record and one
// one-record LOOP with the summed count: the same operations in the same
// order, run by the kernels as a register loop with the constants loaded
// once instead of one table record per repetition.
void fk::merge_repeats(std::vector<OpRec> &ops)
{
    const size_t n = ops.size();
    std::vector<char> in_body(n, 0);
    for (size_t k = 0; k < n; ++k)
        if (ops[k].code == OPC_LOOP && ops[k].span > 1)
            for (size_t j = k - (size_t)ops[k].span; j < k; ++j)
                in_body[j] = 1;
    std::vector<OpRec> out;
    out.reserve(n);
    size_t k = 0;
    while (k < n) {
        if (ops[k].code == OPC_LOOP || in_body[k]) {
            out.push_back(ops[k]);
            ++k;
            continue;
        }
        const OpRec r = ops[k];
        int64_t total = 0;
        size_t j = k;
        while (j < n && ops[j].code != OPC_LOOP && !in_body[j] && same_record(ops[j], r)) {
            int64_t c = 1;
            size_t next = j + 1;
            if (next < n && ops[next].code == OPC_LOOP && ops[next].span == 1) {
                c = ops[next].count;
                ++next;
            }
            if (total + c > INT32_MAX)
                break;
            total += c;
            j = next;
        }
        out.push_back(r);
        if (total > 1) {
            OpRec l;
            std::memset(&l, 0, sizeof l);
            l.code = OPC_LOOP;
            l.span = 1;
            l.count = (int32_t)total;
            out.push_back(l);
        }
        k = j;
    }
    ops.swap(out);
}

// Runs of each record code when the list executes, loops unrolled
// (cnt[OPC_MUL .. OPC_FMA]; LOOP records themselves are not counted).
void fk::executed_counts(const std::vector<OpRec> &ops, double cnt[4])
{
    for (int c = 0; c < 4; ++c)
        cnt[c] = 0.0;
    std::vector<double> times(ops.size(), 1.0);
    for (size_t k = 0; k < ops.size(); ++k)
        if (ops[k].code == OPC_LOOP)
            for (size_t j = k - (size_t)ops[k].span; j < k; ++j)
                times[j] = ops[k].count;
    for (size_t k = 0; k < ops.size(); ++k)
        if (ops[k].code != OPC_LOOP)
            cnt[ops[k].code] += times[k];
}

// Compile-time chains built into the library.
int fk::match_static(const fk_chain_desc *ch, std::vector<float> &consts, int &n_ops)
{
    const fk_op_desc *o = ch->ops;
    // crop+resize u8x3 -> swap, cvt, mul(1), sub, div -> planar f32
    if (ch->read.kind == FK_READ_CROP_RESIZE && ch->read.in_dtype == FK_U8 &&
        ch->read.channels == 3 && ch->write.out_dtype == FK_F32 && ch->write.layout == FK_PLANAR &&
        ch->n_ops == 5 && o[0].kind == FK_OP_SWAP_RB && o[1].kind == FK_OP_CVT_F32 &&
        o[2].kind == FK_OP_MUL && o[2].n_consts == 1 && o[3].kind == FK_OP_SUB &&
        o[4].kind == FK_OP_DIV) {
        consts.assign(7, 0.0f);
        consts[0] = o[2].consts[0];
        for (int c = 0; c < 3; ++c) {
            consts[1 + c] = o[3].n_consts == 1 ? o[3].consts[0] : o[3].consts[c];
            consts[4 + c] = o[4].n_consts == 1 ? o[4].consts[0] : o[4].consts[c];
        }
        n_ops = 5;
        return FAM_NORMALIZE;
    }
    // plain u8x3 -> cvt, N alternating mul/add (scalar) -> packed f32
    if (ch->read.kind == FK_READ_PLAIN && ch->read.in_dtype == FK_U8 && ch->read.channels == 3 &&
        ch->write.out_dtype == FK_F32 && ch->write.layout == FK_PACKED && ch->n_ops >= 2 &&
        o[0].kind == FK_OP_CVT_F32) {
        const int N = ch->n_ops - 1;
        bool ok = N == 1 || N == 4 || N == 16 || N == 64 || N == 256;
        for (int k = 0; ok && k < N; ++k) {
            const fk_op_desc &d = o[1 + k];
            ok = d.kind == (k % 2 == 0 ? FK_OP_MUL : FK_OP_ADD) && d.n_consts == 1;
        }
        if (ok) {
            consts.assign(N, 0.0f);
            for (int k = 0; k < N; ++k)
                consts[k] = o[1 + k].consts[0];
            n_ops = N;
            return FAM_MULADD;
        }
    }
    // plain u8 or fp32 (1 or 3 channels) -> [cvt,] mul, add (scalar), loop over
    // both -> packed f32
    if (ch->read.kind == FK_READ_PLAIN &&
        (ch->read.in_dtype == FK_U8 || ch->read.in_dtype == FK_F32) &&
        (ch->read.channels == 1 || ch->read.channels == 3) && ch->write.out_dtype == FK_F32 &&
        ch->write.layout == FK_PACKED && ch->n_ops >= 3) {
        const fk_op_desc *q = o[0].kind == FK_OP_CVT_F32 ? o + 1 : o;
        if (ch->n_ops == (int)(q - o) + 3 && q[0].kind == FK_OP_MUL && q[0].n_consts == 1 &&
            q[1].kind == FK_OP_ADD && q[1].n_consts == 1 && q[2].kind == FK_OP_LOOP &&
            q[2].loop_span == 2) {
            consts.assign(2, 0.0f);
            consts[0] = q[0].consts[0];
            consts[1] = q[1].consts[0];
            n_ops = q[2].loop_count;
            return FAM_MULADD_LOOP;
        }
    }
    return FAM_RUNTIME;
}
