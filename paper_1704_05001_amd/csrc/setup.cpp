// Hierarchy build (host orchestration of the setup kernels).
//
// Per level (sections 4.1, 5.1, 5.2 of the paper):
//   block sizes and block-diagonal inverses -> strength -> C/F splitting ->
//   coarse numbering -> one-point interpolation -> Neumann restriction
//   Z = -(sum_{i<=k} A_cf T^i) D_ff^{-1} with T = -D_ff^{-1} A_ff^phi ->
//   R A by SpGEMM -> K = (R A) P through the one-point map, drop filter.
// The coarsest level (or a level whose splitting stalls) is inverted densely.
//
// A batched hierarchy holds independent systems side by side (contiguous block
// ranges, no coupling): every step above is local to a system's blocks, the
// splitting hashes use indices within the system, and a system that reaches
// its coarsest size is inverted densely on that level while the others go on
// coarsening, so each system's hierarchy equals the one it would get alone.
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <initializer_list>
#include <utility>

#include "hier.h"

namespace nair {
namespace {

constexpr int kRoundBatch = 8;
constexpr int kMaxRounds = 4096;
constexpr int kNoSingular = 0x7f7f7f7f;   // memset(0x7f) pattern

void alloc_vectors(Level &L, int bs) {
    const size_t n = static_cast<size_t>(L.A.nb) * bs;
    L.r.alloc(n);
    L.e0.alloc(n);
    L.e1.alloc(n);
    L.tmp.alloc(n);
}

// Device copies of the per-system offsets and modes (batches only: one
// system's kernels never read them).
void upload_systems(Level &L, hipStream_t s) {
    const int nsys = static_cast<int>(L.mode.size());
    if (nsys == 1) return;
    if (!L.seg_d.get()) L.seg_d.alloc(nsys + 1);
    if (!L.mode_d.get()) L.mode_d.alloc(nsys);
    NAIR_HIP(hipMemcpyAsync(L.seg_d.get(), L.seg.data(), sizeof(int) * (nsys + 1), hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(L.mode_d.get(), L.mode.data(), nsys, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipStreamSynchronize(s));   // seg and mode may change on the host afterwards
}

// Dense inverses of the systems solved directly on this level (mode 2).
void make_direct(Level &L, int lvl, hipStream_t s) {
    const int bs = L.A.bs;
    L.dsys.clear();
    L.dblk0.clear();
    L.dnb.clear();
    L.doff.clear();
    int64_t off = 0;
    L.dmax_n = 0;
    for (size_t k = 0; k < L.mode.size(); ++k)
        if (L.mode[k] == 2) {
            const int nbk = L.seg[k + 1] - L.seg[k];
            const int64_t n = static_cast<int64_t>(nbk) * bs;
            L.dsys.push_back(static_cast<int>(k));
            L.dblk0.push_back(L.seg[k]);
            L.dnb.push_back(nbk);
            L.doff.push_back(off);
            off += n * n;
            L.dmax_n = std::max(L.dmax_n, static_cast<int>(n));
        }
    L.ndseg = static_cast<int>(L.dsys.size());
    if (L.ndseg == 0) return;
    L.dense_n = (L.ndseg == 1 && L.dnb[0] == L.A.nb) ? L.A.nb * bs : 0;
    L.dense_inv.alloc(static_cast<size_t>(off));
    L.dense_invT.alloc(static_cast<size_t>(off));
    const int bad = dense_inverse_segments(L.A, L.ndseg, L.dblk0.data(), L.dnb.data(), L.doff.data(),
                                           L.dense_inv.get(), L.dense_invT.get(), s);
    if (bad >= 0)
        fail(NAIR_ESINGULAR, "coarsest operator of system " + std::to_string(L.dsys[bad]) + " (level " +
                                 std::to_string(lvl) + ", " + std::to_string(L.dnb[bad] * bs) +
                                 " unknowns) is singular");
    std::vector<int> dof0(L.ndseg), nn(L.ndseg);
    for (int k = 0; k < L.ndseg; ++k) {
        dof0[k] = L.dblk0[k] * bs;
        nn[k] = L.dnb[k] * bs;
    }
    L.ddof0_d.alloc(L.ndseg);
    L.dn_d.alloc(L.ndseg);
    L.dsys_d.alloc(L.ndseg);
    L.doff_d.alloc(L.ndseg);
    NAIR_HIP(hipMemcpyAsync(L.dsys_d.get(), L.dsys.data(), sizeof(int) * L.ndseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(L.ddof0_d.get(), dof0.data(), sizeof(int) * L.ndseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(L.dn_d.get(), nn.data(), sizeof(int) * L.ndseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipMemcpyAsync(L.doff_d.get(), L.doff.data(), sizeof(int64_t) * L.ndseg, hipMemcpyHostToDevice, s));
    NAIR_HIP(hipStreamSynchronize(s));   // dof0 and nn are pageable host memory
}

// C/F splitting by independent-set rounds; state ends as 1 (C) / 0 (F) in L.cf.
// After each batch of rounds `enqueue` launches work whose results `extra`
// reads back with the round counts (the last batch's are what the caller gets).
void split(Hier &h, Level &L, int lvl, hipStream_t s, const std::function<void()> &enqueue,
           const std::vector<ReadItem> &extra) {
    const int n = L.A.nb;
    const int64_t nz = L.A.bound();
    DBuf<int> stptr(static_cast<size_t>(n) + 1), fill(n), stidx(nz > 0 ? nz : 1);
    DBuf<int8_t> newc(n);
    DBuf<int> counts(kMaxRounds + 1);
    launch_fill_ints({{fill.get(), n, 0}, {counts.get(), kMaxRounds + 1, 0}}, s);
    scan_exclusive(L.lambda.get(), stptr.get(), n, s);
    launch_strong_transpose(L.A.rowptr.get(), L.A.colidx.get(), L.mask.get(), n, stptr.get(), fill.get(),
                            stidx.get(), s);
    launch_pmis_init(L.lambda.get(), L.direct.get(), n, L.cf.get(), L.dround.get(), counts.get(), s);
    // rounds go out kRoundBatch at a time (a round after the last one with undecided
    // blocks returns at once), then one read of the counts before and after each
    L.rounds = 0;
    int r = 0;
    while (true) {
        const int first = r;
        for (int b = 0; b < kRoundBatch; ++b) {
            ++r;
            launch_pmis_round(L.A.rowptr.get(), L.A.colidx.get(), L.mask.get(), stptr.get(), stidx.get(),
                              L.lambda.get(), L.lbase.get(), n, h.prm.seed, lvl, r, L.cf.get(), newc.get(),
                              L.dround.get(), counts.get() + r, s);
        }
        int hc[kRoundBatch + 1];
        enqueue();
        std::vector<ReadItem> items{{counts.get() + first, hc, sizeof(hc)}};
        items.insert(items.end(), extra.begin(), extra.end());
        read_device(items.data(), items.size(), s);
        for (int b = 0; b <= kRoundBatch; ++b)
            if (hc[b] == 0) {
                L.rounds = first + b;   // 0: nothing was undecided at the start
                return;
            }
        if (r + kRoundBatch > kMaxRounds) fail(NAIR_ECOARSEN, "splitting did not finish");
    }
}

}  // namespace

void build_hierarchy(Hier &h, int nsys, const int *sys_nb, int nb, int bs, const int *rowptr, const int *colidx,
                     const double *vals, hipStream_t s) {
    const nair_params &p = h.prm;
    h.bs = bs;
    h.bs0 = bs;
    h.nsys = nsys;
    int bb = bs * bs;
    const int nnzb = read_int(rowptr + nb, s);
    if (nnzb < nb) fail(NAIR_EINVAL, "rowptr[nb] < nb: every row needs its diagonal block");
    auto L0 = std::make_unique<Level>();
    L0->seg.assign(nsys + 1, 0);
    for (int k = 0; k < nsys; ++k) L0->seg[k + 1] = L0->seg[k] + sys_nb[k];
    L0->mode.assign(nsys, 0);
    upload_systems(*L0, s);
    {
        DBuf<int> bad(1);
        NAIR_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), s));
        launch_validate(rowptr, colidx, nb, nnzb, nsys > 1 ? L0->seg_d.get() : nullptr, nsys, bad.get(), s);
        const int vb = read_int(bad.get(), s);
        if (vb & 1) fail(NAIR_EINVAL, "rowptr is not a non-decreasing offset array from 0 to nnzb");
        if (vb & 2) fail(NAIR_EINVAL, "column index out of range");
        if (vb & 4) fail(NAIR_EINVAL, "block columns of a row are not strictly increasing");
        if (vb & 8) fail(NAIR_EINVAL, "a row has no diagonal block");
        if (vb & 16) fail(NAIR_EINVAL, "a block couples two systems of the batch");
    }
    DevBSR &Ain = (p.form == 1) ? h.A0 : L0->A;   // the caller's system
    Ain.alloc(nb, nb, bs, nnzb);
    NAIR_HIP(hipMemcpyAsync(Ain.rowptr.get(), rowptr, sizeof(int) * (static_cast<size_t>(nb) + 1),
                            hipMemcpyDeviceToDevice, s));
    NAIR_HIP(hipMemcpyAsync(Ain.colidx.get(), colidx, sizeof(int) * static_cast<size_t>(nnzb),
                            hipMemcpyDeviceToDevice, s));
    // (block form: the values are copied by the first pass over them, the finest level's block sizes)
    const double *copy_from = p.form == 1 ? nullptr : vals;   // (null once copied)
    if (!copy_from)
        NAIR_HIP(hipMemcpyAsync(Ain.vals.get(), vals, sizeof(double) * static_cast<size_t>(nnzb) * bb,
                                hipMemcpyDeviceToDevice, s));
    if (p.form == 1) {
        // scalar form: D^{-1} of the caller's blocks, S = D^{-1} A as the scalar level 0
        h.d0inv.alloc(static_cast<size_t>(nb) * bb);
        DBuf<int> sing(1);
        NAIR_HIP(hipMemsetAsync(sing.get(), 0x7f, sizeof(int), s));
        launch_block_inverse(h.A0.rowptr.get(), h.A0.colidx.get(), h.A0.vals.get(), nb, bs, nullptr, h.d0inv.get(),
                             sing.get(), s);
        const int hs = read_int(sing.get(), s);
        if (hs != kNoSingular)
            fail(NAIR_ESINGULAR, "diagonal block " + std::to_string(hs) + " of the system is singular");
        if (nsys > 1) {
            h.bsys0.alloc(nb);
            launch_seg_info(L0->seg_d.get(), L0->mode_d.get(), nsys, nb, nullptr, nullptr, h.bsys0.get(), s);
        }
        build_scaled(h.A0, h.d0inv.get(), L0->A, s);
        h.rres.alloc(static_cast<size_t>(nb) * bs);
        for (auto &o : L0->seg) o *= bs;   // systems in scalar rows
        bs = 1;
        bb = 1;
        h.bs = 1;
    }
    h.lv.push_back(std::move(L0));

    for (int l = 0;; ++l) {
        Level &L = *h.lv[l];
        const int n = L.A.nb;
        g_timer_level = l;
        alloc_vectors(L, bs);
        // systems at their coarsest size (or the last allowed level) are solved directly here
        int ncont = 0, ndir = 0;
        for (int k = 0; k < nsys; ++k) {
            const int len = L.seg[k + 1] - L.seg[k];
            if (len == 0) {
                L.mode[k] = 0;
            } else if (static_cast<int64_t>(len) * bs <= p.max_coarse_dofs || l == p.max_levels - 1) {
                L.mode[k] = 2;
                ++ndir;
            } else {
                L.mode[k] = 1;
                ++ncont;
            }
        }
        upload_systems(L, s);
        if (nsys > 1) {
            L.bsys.alloc(n);
            if (ncont > 0) L.lbase.alloc(n);
            if (ncont > 0 && ndir > 0) L.direct.alloc(n);
            launch_seg_info(L.seg_d.get(), L.mode_d.get(), nsys, n, L.lbase.get(), L.direct.get(), L.bsys.get(), s);
        }
        if (ncont == 0) {
            if (copy_from) {   // solved directly at the finest level: no pass over the values to copy them
                NAIR_HIP(hipMemcpyAsync(L.A.vals.get(), copy_from, sizeof(double) * static_cast<size_t>(nnzb) * bb,
                                        hipMemcpyDeviceToDevice, s));
                copy_from = nullptr;
            }
            if (L.A.nnzb < 0) L.A.nnzb = read_int(L.A.rowptr.get() + n, s);
            L.coarsest = true;
            make_direct(L, l, s);
            break;
        }
        const int64_t nz = L.A.bound();   // (the exact count comes back with the splitting's read)
        L.dinv.alloc(static_cast<size_t>(n) * bb);
        if (!L.bnorm_ready) L.bnorm.alloc(nz);
        L.mask.alloc(nz);
        L.lambda.alloc(n);
        L.cf.alloc(n);
        L.cidx.alloc(n);
        L.pmap.alloc(n);
        L.dround.alloc(n);
        DBuf<int> sing(1);
        L.margin.alloc(4);
        launch_fill_ints({{sing.get(), 1, kNoSingular}, {L.lambda.get(), n, 0}, {L.margin.get(), 4, 0}}, s);
        if (!L.bnorm_ready) {
            if (l == 0 && copy_from) {   // the caller's values: copied here; the face copy's masks come along
                if (p.faces == 1) L.facemeta.alloc(static_cast<size_t>(nz));
                launch_block_scan(copy_from, nz, bs, nullptr, nullptr, L.bnorm.get(), L.facemeta.get(), nullptr,
                                  nullptr, s, L.A.vals.get());
                copy_from = nullptr;
            } else {
                launch_block_maxabs(L.A.vals.get(), nz, bs, L.bnorm.get(), s);
            }
        }
        {
            TimerScope ts(TK_BLOCKINV, l, s);
            launch_block_inverse(L.A.rowptr.get(), L.A.colidx.get(), L.A.vals.get(), n, bs, L.direct.get(),
                                 L.dinv.get(), sing.get(), s);
        }
        launch_strength(L.A.rowptr.get(), L.A.colidx.get(), L.bnorm.get(), n, p.theta, p.phi, L.mask.get(),
                        L.lambda.get(), L.margin.get(), s);
        if (l == 0 && p.cf_override_host) {
            std::vector<int8_t> cfh(n);
            for (int I = 0; I < n; ++I) cfh[I] = p.cf_override_host[I] ? 1 : 0;
            NAIR_HIP(hipMemcpyAsync(L.cf.get(), cfh.data(), n, hipMemcpyHostToDevice, s));
            NAIR_HIP(hipMemsetAsync(L.dround.get(), 0, sizeof(int) * n, s));
            if (L.direct.get()) launch_mark_direct(L.direct.get(), n, L.cf.get(), s);
            NAIR_HIP(hipStreamSynchronize(s));   // cfh is pageable host memory
            L.rounds = 0;
        }
        // coarse blocks per system (as offsets) and the singular flag: counted on the
        // device after the splitting and read back with its last round counts
        DBuf<int> cflag(n), cscan(static_cast<size_t>(n) + 1);
        std::vector<int> cseg(nsys + 2);   // coarse blocks per system, as offsets; then the singular flag
        DBuf<int> cseg_d(nsys + 2);
        cseg[0] = 0;
        auto count_c_launch = [&]() {
            launch_cf_flags(L.cf.get(), n, 1, cflag.get(), s);
            scan_exclusive(cflag.get(), cscan.get(), n, s);
            if (nsys == 1) return;   // one system: its C count is the scan's total
            launch_gather_int(cscan.get(), L.seg_d.get(), nsys + 1, cseg_d.get(), s);
            NAIR_HIP(hipMemcpyAsync(cseg_d.get() + nsys + 1, sing.get(), sizeof(int), hipMemcpyDeviceToDevice, s));
        };
        const std::vector<ReadItem> count_c_items =
            nsys == 1 ? std::vector<ReadItem>{{cscan.get() + n, &cseg[1], sizeof(int)},
                                              {sing.get(), &cseg[2], sizeof(int)}}
                      : std::vector<ReadItem>{{cseg_d.get(), cseg.data(), sizeof(int) * (nsys + 2)}};
        auto count_c = [&]() {
            count_c_launch();
            read_device(count_c_items.data(), count_c_items.size(), s);
        };
        int anz = 0;
        std::vector<ReadItem> split_items = count_c_items;
        if (L.A.nnzb < 0) split_items.push_back({L.A.rowptr.get() + n, &anz, sizeof(int)});
        if (l == 0 && p.cf_override_host) count_c();
        else split(h, L, l, s, count_c_launch, split_items);
        if (L.A.nnzb < 0) L.A.nnzb = anz;
        const int hsing = cseg[nsys + 1];
        if (hsing != kNoSingular)
            fail(NAIR_ESINGULAR, "diagonal block " + std::to_string(hsing) + " of level " + std::to_string(l) +
                                     " is singular");
        // a system whose splitting stalls (no C or no F block) is solved directly here
        bool stalled = false;
        for (int k = 0; k < nsys; ++k) {
            if (L.mode[k] != 1) continue;
            const int len = L.seg[k + 1] - L.seg[k];
            const int nck = cseg[k + 1] - cseg[k];
            if (nck != 0 && nck != len) continue;
            if (static_cast<int64_t>(len) * bs > kStallDenseDofs)
                fail(NAIR_ECOARSEN, "splitting of level " + std::to_string(l) + " (" + std::to_string(len) +
                                        " blocks" + (nsys > 1 ? ", system " + std::to_string(k) : std::string()) +
                                        ") gave " + std::to_string(nck) + " C blocks");
            L.mode[k] = 2;
            --ncont;
            ++ndir;
            stalled = true;
        }
        if (stalled) {
            upload_systems(L, s);
            if (ncont == 0) {
                L.coarsest = true;
                make_direct(L, l, s);
                break;
            }
            if (!L.direct.get()) L.direct.alloc(n);
            launch_seg_info(L.seg_d.get(), L.mode_d.get(), nsys, n, nullptr, L.direct.get(), nullptr, s);
            launch_mark_direct(L.direct.get(), n, L.cf.get(), s);
            count_c();
        }
        if (ndir > 0) make_direct(L, l, s);
        const int nc = cseg[nsys];
        L.nc = nc;
        DBuf<int> fscan;
        if (ndir > 0) {
            fscan.alloc(static_cast<size_t>(n) + 1);
            launch_cf_flags(L.cf.get(), n, 0, cflag.get(), s);
            scan_exclusive(cflag.get(), fscan.get(), n, s);
            L.nF = read_int(fscan.get() + n, s);
        } else {
            L.nF = n - nc;
        }
        L.cpts.alloc(nc);
        L.flist.alloc(L.nF);
        launch_cf_index(L.cf.get(), cscan.get(), fscan.get(), n, L.cidx.get(), L.cpts.get(), L.flist.get(), s);
        launch_one_point(L.A.rowptr.get(), L.A.colidx.get(), L.bnorm.get(), L.cf.get(), L.cidx.get(), n,
                         L.pmap.get(), L.margin.get(), s);
        // Neumann operands: T (phi-strong F-F, scaled by -D_ff^{-1}) and W_0 = A_cf
        DevBSR T, W0;
        T.nb = n;
        T.ncols = n;
        T.bs = bs;
        T.rowptr.alloc(static_cast<size_t>(n) + 1);
        W0.nb = nc;
        W0.ncols = n;
        W0.bs = bs;
        W0.rowptr.alloc(static_cast<size_t>(nc) + 1);
        int tot[2] = {0, 0};   // blocks of T and of W_0, side by side for one copy
        {
            DBuf<int> cntT(n), cntW(nc), dtot(2);
            launch_count_T(L.A.rowptr.get(), L.A.colidx.get(), L.mask.get(), L.cf.get(), n, cntT.get(), s);
            launch_count_Acf(L.A.rowptr.get(), L.A.colidx.get(), L.cf.get(), L.cpts.get(), nc, cntW.get(), s);
            scan_exclusive2(cntT.get(), T.rowptr.get(), n, dtot.get(), cntW.get(), W0.rowptr.get(), nc, dtot.get() + 1,
                            s);
            read_ints(dtot.get(), tot, 2, s);
        }
        const int nT = tot[0], nW = tot[1];
        T.nnzb = nT;
        T.colidx.alloc(nT);
        T.vals.alloc(static_cast<size_t>(nT) * bb);
        {
            DBuf<int> trow(nT), tsrc(nT);
            launch_fill_T(L.A.rowptr.get(), L.A.colidx.get(), L.mask.get(), L.cf.get(), n, T.rowptr.get(),
                          T.colidx.get(), trow.get(), tsrc.get(), s);
            TimerScope ts(TK_BLOCKPROD, l, s);
            launch_block_product(nT, bs, L.dinv.get(), trow.get(), L.A.vals.get(), tsrc.get(), -1.0, T.vals.get(),
                                 s);
        }
        // (on the matrix cores W_0 keeps no values of its own: its block t is A's block wsrc[t])
        const bool masks = use_matrix_cores(bs);   // the matrix-core products give each block's nonzero rows
        W0.nnzb = nW;
        W0.colidx.alloc(nW);
        DBuf<int> wsrc(nW);
        launch_fill_Acf(L.A.rowptr.get(), L.A.colidx.get(), L.cf.get(), L.cpts.get(), nc, W0.rowptr.get(),
                        W0.colidx.get(), wsrc.get(), s);
        if (!masks) {
            W0.vals.alloc(static_cast<size_t>(nW) * bb);
            launch_block_gather(nW, bs, L.A.vals.get(), wsrc.get(), W0.vals.get(), s);
        }
        // S = ((W_0 + W_1) + W_2) + ...,  W_i = W_{i-1} T.  On the matrix cores S
        // is not stored: its pattern comes with one map per term (term i's block
        // of each S block, or -1), and Z's product below adds the terms itself.
        const bool fused_sum = masks && p.degree >= 1;
        std::vector<DevBSR> terms;   // W_0 .. W_k (fused) or the last W (stored sums)
        std::vector<DBuf<int>> tmaps;
        terms.push_back(std::move(W0));
        DevBSR S;
        bool s_is_w0 = true;
        for (int d = 1; d <= p.degree; ++d) {
            DevBSR Wd;
            if (masks && d == 1)
                spgemm(terms[0], nullptr, T, Wd, s, L.A.vals.get(), wsrc.get());
            else
                spgemm(terms.back(), nullptr, T, Wd, s);
            DevBSR Snew;
            if (fused_sum) {
                DBuf<int> mS, mW;
                bsr_add(s_is_w0 ? terms[0] : S, Wd, Snew, s, &mS, &mW);
                if (d == 1 || !mS.get()) {   // (no blocks: maps stay empty)
                    tmaps.clear();
                    tmaps.push_back(std::move(mS));
                } else {
                    compose_term_maps(Snew.bound(), Snew.rowptr.get() + nc, mS.get(), tmaps, s);
                }
                tmaps.push_back(std::move(mW));
                terms.push_back(std::move(Wd));
            } else {
                bsr_add(s_is_w0 ? terms[0] : S, Wd, Snew, s);
                terms.back() = std::move(Wd);
            }
            S = std::move(Snew);
            s_is_w0 = false;
        }
        DevBSR &Ssum = s_is_w0 ? terms[0] : S;
        // Z_IJ = -(S_IJ Dinv_J)
        L.Z.nb = nc;
        L.Z.ncols = n;
        L.Z.bs = bs;
        L.Z.nnzb = Ssum.nnzb;   // (on the device when S is a sum; the Galerkin step reads it back)
        L.Z.cap = Ssum.bound();
        L.Z.rowptr = std::move(Ssum.rowptr);
        L.Z.colidx = std::move(Ssum.colidx);
        L.Z.vals.alloc(static_cast<size_t>(L.Z.cap) * bb);
        if (masks) L.zmask.alloc(static_cast<size_t>(L.Z.cap));
        {
            TimerScope ts(TK_BLOCKPROD, l, s);
            const int *zcount = L.Z.nnzb < 0 ? L.Z.rowptr.get() + nc : nullptr;
            if (fused_sum) {
                if (L.Z.cap > 0) {
                    // term 0 (W_0) is read from A's blocks
                    launch_map_through(L.Z.cap, zcount, tmaps[0].get(), wsrc.get(), s);
                    SumTerms st;
                    st.n = static_cast<int>(terms.size());
                    for (int i = 0; i < st.n; ++i) {
                        st.vals[i] = i == 0 ? L.A.vals.get() : terms[i].vals.get();
                        st.map[i] = tmaps[i].get();
                    }
                    launch_sum_product(L.Z.cap, bs, st, L.dinv.get(), L.Z.colidx.get(), -1.0, L.Z.vals.get(), s,
                                       zcount, L.zmask.get());
                }
            } else if (masks) {   // degree 0: Z = -(W_0 D^-1) with W_0's blocks read from A
                launch_block_product(L.Z.cap, bs, L.A.vals.get(), wsrc.get(), L.dinv.get(), L.Z.colidx.get(), -1.0,
                                     L.Z.vals.get(), s, zcount, L.zmask.get());
            } else {
                launch_block_product(L.Z.cap, bs, Ssum.vals.get(), nullptr, L.dinv.get(), L.Z.colidx.get(), -1.0,
                                     L.Z.vals.get(), s, zcount, nullptr);
            }
        }
        // Galerkin: K = R A P with R = [Z I], filtered; K's block sizes come along
        auto next = std::make_unique<Level>();
        galerkin(L.Z, L.cpts.get(), L.A, L.pmap.get(), nc, p.drop, next->A, L.margin.get(), next->bnorm,
                 next->amask, s);
        next->bnorm_ready = true;
        next->seg.assign(cseg.begin(), cseg.begin() + nsys + 1);
        next->mode.assign(nsys, 0);
        h.lv.push_back(std::move(next));
    }
    // the finest operator is read by every cycle: a compact copy of its face blocks
    if (p.faces == 1 && p.form == 0) build_face(h.lv[0]->A, h.lv[0]->face, s, &h.lv[0]->facemeta);
    build_sweeps(h, false, s);
    if (p.precision == 1) make_fp32_copies(h, s);
    prepare_cycle(h, false, s);   // the F-cycle's saved vectors
    NAIR_HIP(hipStreamSynchronize(s));
}

void build_sweeps(Hier &h, bool trans, hipStream_t s) {
    if (h.prm.sweep_copy == 0) return;
    for (auto &Lp : h.lv) {
        Level &L = *Lp;
        if (L.coarsest || L.nF <= 0) continue;
        if (h.prm.sweep_copy < 0 && few_lanes(L.A.nb, L.A.bs)) continue;
        if (trans && (L.atF.on || !L.AT.rowptr.get())) continue;   // the transposed sweeps read A's rows
        SweepCopy &S = trans ? L.sweepT : L.sweep;
        // (A's row masks, where the Galerkin step gave them, are no use for A^T)
        if (!S.on)
            build_sweep(trans ? L.AT : L.A, trans ? L.faceT : L.face, L.dinv.get(), L.flist.get(), L.nF, S, s, trans,
                        trans ? nullptr : L.amask.get());
        if (!trans && !L.zrows.on && L.Z.nnzb > 0)
            build_row_blocks(L.Z.vals.get(), L.Z.nnzb, L.Z.bs, L.zrows, s, nullptr, nullptr, L.zmask.get());
    }
}

// FP32 copies of what the cycle reads (operators and Z of the non-coarsest
// levels, and their transposes once built), plus FP32 cycle vectors.
void make_fp32_copies(Hier &h, hipStream_t s) {
    for (auto &Lp : h.lv) {
        Level &L = *Lp;
        const size_t n = static_cast<size_t>(L.A.nb) * L.A.bs;
        const int64_t bb = static_cast<int64_t>(L.A.bs) * L.A.bs;
        if (!L.r32.get()) {
            L.r32.alloc(n);
            L.e0_32.alloc(n);
            L.e1_32.alloc(n);
            L.tmp32.alloc(n);
        }
        // every level's operator (the F-cycle's coarse solve takes a residual
        // on the coarsest level too); Z only where the level coarsens
        if (!L.vals32.get()) {
            L.vals32.alloc(static_cast<size_t>(L.A.nnzb * bb));
            launch_to_float(L.A.vals.get(), L.vals32.get(), L.A.nnzb * bb, s);
            if (!L.coarsest && !L.zrows.on) {   // (with a row-compressed Z the restriction reads only that)
                L.z32.alloc(static_cast<size_t>(L.Z.nnzb * bb));
                launch_to_float(L.Z.vals.get(), L.z32.get(), L.Z.nnzb * bb, s);
            }
        }
        if (L.have_T && L.AT.rowptr.get() && !L.at32.get()) {
            L.at32.alloc(static_cast<size_t>(L.AT.nnzb * bb));
            launch_to_float(L.AT.vals.get(), L.at32.get(), L.AT.nnzb * bb, s);
        }
        if (L.have_T && !L.coarsest && L.ZT.rowptr.get() && !L.zt32.get()) {
            L.zt32.alloc(static_cast<size_t>(L.ZT.nnzb * bb));
            launch_to_float(L.ZT.vals.get(), L.zt32.get(), L.ZT.nnzb * bb, s);
        }
        face_to_float(L.A, L.face, s);
        if (L.have_T) face_to_float(L.AT, L.faceT, s);
        trans_rows_to_float(L.atF, L.A.bs, s);
        trans_rows_to_float(L.zt, L.A.bs, s);
        sweep_to_float(L.sweep, L.A.bs, s);
        sweep_to_float(L.sweepT, L.A.bs, s);
        row_blocks_to_float(L.zrows, L.Z.nnzb, L.A.bs, s);
    }
}

void ensure_transposes(Hier &h, hipStream_t s) {
    if (h.prm.form == 1 && !h.have_A0T) {   // the transposed outer residual uses A0^T
        bsr_transpose(h.A0, h.A0T, s);
        h.have_A0T = true;
    }
    for (size_t l = 0; l < h.lv.size(); ++l) {
        Level &L = *h.lv[l];
        if (L.have_T) continue;
        // below the finest level, the transposed sweeps and residual read A's
        // rows transposed by their nonzero rows (only the F rows: with F
        // relaxation the transposed sweeps leave y zero on C rows); the finest
        // level reads A^T (its face copy, or its sweep copy), as the forward
        // cycle reads A, whether or not it is face-shaped
        const bool rows_tr = L.A.bs >= 4 && !L.coarsest;
        if (rows_tr && l > 0)
            build_trans_rows(L.A, h.prm.relax == 1 ? nullptr : L.cf.get(), 0, L.amask.get(), L.atF, s);
        // A^T itself: the finest level (face copy, outer residual), the F-cycle's
        // coarse residuals, small blocks and the coarsest level
        if (!L.atF.on || l == 0 || h.prm.cycle == 1) {
            bsr_transpose(L.A, L.AT, s);
            if (L.face.on) build_face(L.AT, L.faceT, s);   // A^T's blocks have the transposed faces
        }
        if (!L.coarsest) {
            if (rows_tr) build_trans_rows(L.Z, nullptr, 0, L.zmask.get(), L.zt, s);
            if (!L.zt.on) bsr_transpose(L.Z, L.ZT, s);
            pmap_transpose(L.pmap.get(), L.A.nb, L.nc, L.ptptr, L.ptidx, s);
        }
        L.have_T = true;
    }
    build_sweeps(h, true, s);
    if (h.prm.precision == 1) make_fp32_copies(h, s);
    NAIR_HIP(hipStreamSynchronize(s));
}

void complexity(Hier &h, double *oc, double *cc, hipStream_t s) {
    const double nnz0 = static_cast<double>(h.lv[0]->A.nnzb);
    const int nu = h.prm.degree + 1;
    const size_t nl = h.lv.size();
    std::vector<double> w(nl, 0.0), nz(nl, 0.0);   // per-level V-cycle work, operator size
    double o = 0.0;
    for (size_t l = 0; l < nl; ++l) {
        Level &L = *h.lv[l];
        nz[l] = static_cast<double>(L.A.nnzb) / nnz0;
        o += nz[l];
        // dense solves count their n^2 entries in block units
        for (int k = 0; k < L.ndseg; ++k) w[l] += static_cast<double>(L.dnb[k]) * L.dnb[k] / nnz0;
        if (L.coarsest) continue;
        std::vector<int> rp(L.A.nb + 1);
        std::vector<int8_t> cfh(L.A.nb);
        NAIR_HIP(hipMemcpyAsync(rp.data(), L.A.rowptr.get(), sizeof(int) * rp.size(), hipMemcpyDeviceToHost, s));
        NAIR_HIP(hipMemcpyAsync(cfh.data(), L.cf.get(), cfh.size(), hipMemcpyDeviceToHost, s));
        NAIR_HIP(hipStreamSynchronize(s));
        double nzF = 0, nzC = 0, nbF = 0;
        for (int I = 0; I < L.A.nb; ++I) {
            const double rn = rp[I + 1] - rp[I];
            if (cfh[I] == 1) {
                nzC += rn;
            } else if (cfh[I] == 0) {
                nzF += rn;
                nbF += 1;
            }
        }
        w[l] += (nu * nzF + (h.prm.relax == 1 ? nzC : 0.0) + static_cast<double>(L.Z.nnzb) + nbF) / nnz0;
    }
    // V: each level once.  F: a level's coarse solve is an F-cycle, a residual
    // with the coarse operator and a V-cycle, recursively.
    double cv = 0.0, cf = 0.0;
    for (size_t i = nl; i-- > 0;) {
        if (i == nl - 1) {
            cv = w[i];
            cf = w[i];
        } else {
            cf = w[i] + cf + nz[i + 1] + cv;
            cv = w[i] + cv;
        }
    }
    if (oc) *oc = o;
    if (cc) *cc = 1.0 + (h.prm.cycle == 1 ? cf : cv);
}

}  // namespace nair
