// Register-window form of the dedispersion kernel: FP32 input, gfx950, wave64.
//
// Eq. bruteEquation, D[d][t] = sum_c A[c][t + delay(c, d)], over one (512-sample time
// tile, group of 64 DM trials) per workgroup of eight wavefronts. Wavefront w owns trials
// dg + 8w .. dg + 8w + 7; lane l owns output samples t0 + 8l .. t0 + 8l + 7 of each.
//
// Staging. A channel slot holds samples [first, first + xs) of one channel, `first` being
// the delay of the group's first trial: the tile plus the group's delay spread (Eq.
// channelDispersionEquation). The slot holds the samples once, with four words of padding
// after every eight, so that lanes whose windows start eight samples apart read distinct
// LDS banks with ds_read_b128. Slots arrive by 16-byte LDS DMAs through a ring of stages
// of eight channels; each wavefront issues one channel of a stage.
//
// Compute. For each channel a lane reads its window, 4 * NCH consecutive samples starting
// at sample 8l + a of the slot (a = the wavefront's first relative delay rounded down to a
// multiple of eight), into a fixed register range. Trial g then needs window registers
// idx_g .. idx_g + 7, where idx_g = its delay - first - a is the same for every lane: the
// adds run in VGPR index mode (s_set_gpr_idx_on, SRC0 relative to M0), so a staged word
// read once from LDS feeds every trial of the wavefront whose window covers it. The next
// channel's window streams into the other register range while this one is added.
//
// The sums follow the fixed order of the ABI (FP32 in channel order inside blocks of
// DD_CHAN_BLOCK channels, block sums added in order), so the series equal those of the
// four-copy LDS form bit for bit. The FP64 statistics partials of a (trial, tile) sum each
// lane's eight samples in order and then the lanes in a fixed butterfly.
//
// Registers. The compiler keeps to v0..v31 (amdgpu_num_vgpr(16): the attribute counts
// halves of the unified register budget); above that the asm owns:
//   v32..v95    block sums, trial g in v[32 + 8g .. 39 + 8g]
//   v96..v159   running sums, trial g in v[96 + 8g .. 103 + 8g]
//   v160..v207  window A, v208..v255 window B (12 chunks of four samples each)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <string>

#include "dd_internal.h"
#include "dd_device.h"

// The fixed registers above the compiler's share are named in clobber lists so the kernel
// allocates them; clang notes that it does not preserve reserved registers, which is the point.
#pragma clang diagnostic ignored "-Winline-asm"

namespace {

using dd::InView;

constexpr int kRwWaves = 8;  // wavefronts per workgroup
constexpr int kRwG = 8;      // DM trials per wavefront
constexpr int kRwCs = 8;     // channels per stage (one per wavefront for the DMAs)
static_assert(kRwWaves * kRwG == dd::kRwTrials, "trials per group disagree with the host plan");
static_assert(kRwCs == dd::kRwStage, "stage width disagrees with the host plan");

struct RWParams {
  InView in;
  const int32_t* gbase;  // [ngroups][nchan] delay of each group's first trial
  const int4* meta;      // [ngroups][nchan][8]: window byte offset, trial indices 0-3, 4-7
  float* out;
  double* part;          // [ndm][ntiles][2] or null
  int64_t out_stride, nout, nitems;
  int nchan, ndm, ngroups;
  int xs;       // samples one slot's DMAs cover (a multiple of 8)
  int ndma;     // 16-byte DMA instructions per slot; slot bytes = 1024 * ndma
  int nb;       // stages in the LDS ring
  int nstages;  // ceil(nchan / 8)
};

// ---- asm building blocks (register numbers are the map above)
#define RW_ADD(a, w) "v_add_f32 v" #a ", v" #w ", v" #a "\n\t"
#define RW_LD(lo, hi, off) "ds_read_b128 v[" #lo ":" #hi "], %[na] offset:" #off "\n\t"
#define RW_FOLD1(t, s) "v_add_f32 v" #t ", v" #s ", v" #t "\n\tv_mov_b32 v" #s ", 0\n\t"
// trial index g: byte (g & 3) of the packed word; s_bfe_u32 operand = (width 8 << 16) | offset
#define RW_IDX_ON(src, sh) "s_bfe_u32 %[t], %[" #src "], " sh "\n\ts_set_gpr_idx_on %[t], gpr_idx(SRC0)\n\t"
#define RW_IDX(src, sh) "s_bfe_u32 %[t], %[" #src "], " sh "\n\ts_set_gpr_idx_idx %[t]\n\t"
#define RW_B0 "0x80000"
#define RW_B1 "0x80008"
#define RW_B2 "0x80010"
#define RW_B3 "0x80018"

#define RW_TA0 \
  RW_ADD(32, 160) RW_ADD(33, 161) RW_ADD(34, 162) RW_ADD(35, 163) \
  RW_ADD(36, 164) RW_ADD(37, 165) RW_ADD(38, 166) RW_ADD(39, 167)
#define RW_TA1 \
  RW_ADD(40, 160) RW_ADD(41, 161) RW_ADD(42, 162) RW_ADD(43, 163) \
  RW_ADD(44, 164) RW_ADD(45, 165) RW_ADD(46, 166) RW_ADD(47, 167)
#define RW_TA2 \
  RW_ADD(48, 160) RW_ADD(49, 161) RW_ADD(50, 162) RW_ADD(51, 163) \
  RW_ADD(52, 164) RW_ADD(53, 165) RW_ADD(54, 166) RW_ADD(55, 167)
#define RW_TA3 \
  RW_ADD(56, 160) RW_ADD(57, 161) RW_ADD(58, 162) RW_ADD(59, 163) \
  RW_ADD(60, 164) RW_ADD(61, 165) RW_ADD(62, 166) RW_ADD(63, 167)
#define RW_TA4 \
  RW_ADD(64, 160) RW_ADD(65, 161) RW_ADD(66, 162) RW_ADD(67, 163) \
  RW_ADD(68, 164) RW_ADD(69, 165) RW_ADD(70, 166) RW_ADD(71, 167)
#define RW_TA5 \
  RW_ADD(72, 160) RW_ADD(73, 161) RW_ADD(74, 162) RW_ADD(75, 163) \
  RW_ADD(76, 164) RW_ADD(77, 165) RW_ADD(78, 166) RW_ADD(79, 167)
#define RW_TA6 \
  RW_ADD(80, 160) RW_ADD(81, 161) RW_ADD(82, 162) RW_ADD(83, 163) \
  RW_ADD(84, 164) RW_ADD(85, 165) RW_ADD(86, 166) RW_ADD(87, 167)
#define RW_TA7 \
  RW_ADD(88, 160) RW_ADD(89, 161) RW_ADD(90, 162) RW_ADD(91, 163) \
  RW_ADD(92, 164) RW_ADD(93, 165) RW_ADD(94, 166) RW_ADD(95, 167)
#define RW_TB0 \
  RW_ADD(32, 208) RW_ADD(33, 209) RW_ADD(34, 210) RW_ADD(35, 211) \
  RW_ADD(36, 212) RW_ADD(37, 213) RW_ADD(38, 214) RW_ADD(39, 215)
#define RW_TB1 \
  RW_ADD(40, 208) RW_ADD(41, 209) RW_ADD(42, 210) RW_ADD(43, 211) \
  RW_ADD(44, 212) RW_ADD(45, 213) RW_ADD(46, 214) RW_ADD(47, 215)
#define RW_TB2 \
  RW_ADD(48, 208) RW_ADD(49, 209) RW_ADD(50, 210) RW_ADD(51, 211) \
  RW_ADD(52, 212) RW_ADD(53, 213) RW_ADD(54, 214) RW_ADD(55, 215)
#define RW_TB3 \
  RW_ADD(56, 208) RW_ADD(57, 209) RW_ADD(58, 210) RW_ADD(59, 211) \
  RW_ADD(60, 212) RW_ADD(61, 213) RW_ADD(62, 214) RW_ADD(63, 215)
#define RW_TB4 \
  RW_ADD(64, 208) RW_ADD(65, 209) RW_ADD(66, 210) RW_ADD(67, 211) \
  RW_ADD(68, 212) RW_ADD(69, 213) RW_ADD(70, 214) RW_ADD(71, 215)
#define RW_TB5 \
  RW_ADD(72, 208) RW_ADD(73, 209) RW_ADD(74, 210) RW_ADD(75, 211) \
  RW_ADD(76, 212) RW_ADD(77, 213) RW_ADD(78, 214) RW_ADD(79, 215)
#define RW_TB6 \
  RW_ADD(80, 208) RW_ADD(81, 209) RW_ADD(82, 210) RW_ADD(83, 211) \
  RW_ADD(84, 212) RW_ADD(85, 213) RW_ADD(86, 214) RW_ADD(87, 215)
#define RW_TB7 \
  RW_ADD(88, 208) RW_ADD(89, 209) RW_ADD(90, 210) RW_ADD(91, 211) \
  RW_ADD(92, 212) RW_ADD(93, 213) RW_ADD(94, 214) RW_ADD(95, 215)
#define RW_FOLDG0 \
  RW_FOLD1(96, 32) RW_FOLD1(97, 33) RW_FOLD1(98, 34) RW_FOLD1(99, 35) RW_FOLD1(100, 36) RW_FOLD1(101, 37) RW_FOLD1(102, 38) RW_FOLD1(103, 39) RW_FOLD1(104, 40) RW_FOLD1(105, 41) RW_FOLD1(106, 42) RW_FOLD1(107, 43) RW_FOLD1(108, 44) RW_FOLD1(109, 45) RW_FOLD1(110, 46) RW_FOLD1(111, 47)
#define RW_FOLDG1 \
  RW_FOLD1(112, 48) RW_FOLD1(113, 49) RW_FOLD1(114, 50) RW_FOLD1(115, 51) RW_FOLD1(116, 52) RW_FOLD1(117, 53) RW_FOLD1(118, 54) RW_FOLD1(119, 55) RW_FOLD1(120, 56) RW_FOLD1(121, 57) RW_FOLD1(122, 58) RW_FOLD1(123, 59) RW_FOLD1(124, 60) RW_FOLD1(125, 61) RW_FOLD1(126, 62) RW_FOLD1(127, 63)
#define RW_FOLDG2 \
  RW_FOLD1(128, 64) RW_FOLD1(129, 65) RW_FOLD1(130, 66) RW_FOLD1(131, 67) RW_FOLD1(132, 68) RW_FOLD1(133, 69) RW_FOLD1(134, 70) RW_FOLD1(135, 71) RW_FOLD1(136, 72) RW_FOLD1(137, 73) RW_FOLD1(138, 74) RW_FOLD1(139, 75) RW_FOLD1(140, 76) RW_FOLD1(141, 77) RW_FOLD1(142, 78) RW_FOLD1(143, 79)
#define RW_FOLDG3 \
  RW_FOLD1(144, 80) RW_FOLD1(145, 81) RW_FOLD1(146, 82) RW_FOLD1(147, 83) RW_FOLD1(148, 84) RW_FOLD1(149, 85) RW_FOLD1(150, 86) RW_FOLD1(151, 87) RW_FOLD1(152, 88) RW_FOLD1(153, 89) RW_FOLD1(154, 90) RW_FOLD1(155, 91) RW_FOLD1(156, 92) RW_FOLD1(157, 93) RW_FOLD1(158, 94) RW_FOLD1(159, 95)
#define RW_GET0 "v_mov_b32 %0, v96\n\tv_mov_b32 %1, v97\n\tv_mov_b32 %2, v98\n\tv_mov_b32 %3, v99\n\t" \
  "v_mov_b32 %4, v100\n\tv_mov_b32 %5, v101\n\tv_mov_b32 %6, v102\n\tv_mov_b32 %7, v103"
#define RW_GET1 "v_mov_b32 %0, v104\n\tv_mov_b32 %1, v105\n\tv_mov_b32 %2, v106\n\tv_mov_b32 %3, v107\n\t" \
  "v_mov_b32 %4, v108\n\tv_mov_b32 %5, v109\n\tv_mov_b32 %6, v110\n\tv_mov_b32 %7, v111"
#define RW_GET2 "v_mov_b32 %0, v112\n\tv_mov_b32 %1, v113\n\tv_mov_b32 %2, v114\n\tv_mov_b32 %3, v115\n\t" \
  "v_mov_b32 %4, v116\n\tv_mov_b32 %5, v117\n\tv_mov_b32 %6, v118\n\tv_mov_b32 %7, v119"
#define RW_GET3 "v_mov_b32 %0, v120\n\tv_mov_b32 %1, v121\n\tv_mov_b32 %2, v122\n\tv_mov_b32 %3, v123\n\t" \
  "v_mov_b32 %4, v124\n\tv_mov_b32 %5, v125\n\tv_mov_b32 %6, v126\n\tv_mov_b32 %7, v127"
#define RW_GET4 "v_mov_b32 %0, v128\n\tv_mov_b32 %1, v129\n\tv_mov_b32 %2, v130\n\tv_mov_b32 %3, v131\n\t" \
  "v_mov_b32 %4, v132\n\tv_mov_b32 %5, v133\n\tv_mov_b32 %6, v134\n\tv_mov_b32 %7, v135"
#define RW_GET5 "v_mov_b32 %0, v136\n\tv_mov_b32 %1, v137\n\tv_mov_b32 %2, v138\n\tv_mov_b32 %3, v139\n\t" \
  "v_mov_b32 %4, v140\n\tv_mov_b32 %5, v141\n\tv_mov_b32 %6, v142\n\tv_mov_b32 %7, v143"
#define RW_GET6 "v_mov_b32 %0, v144\n\tv_mov_b32 %1, v145\n\tv_mov_b32 %2, v146\n\tv_mov_b32 %3, v147\n\t" \
  "v_mov_b32 %4, v148\n\tv_mov_b32 %5, v149\n\tv_mov_b32 %6, v150\n\tv_mov_b32 %7, v151"
#define RW_GET7 "v_mov_b32 %0, v152\n\tv_mov_b32 %1, v153\n\tv_mov_b32 %2, v154\n\tv_mov_b32 %3, v155\n\t" \
  "v_mov_b32 %4, v156\n\tv_mov_b32 %5, v157\n\tv_mov_b32 %6, v158\n\tv_mov_b32 %7, v159"
#define RW_CLOB_SUB \
  "v32", "v33", "v34", "v35", "v36", "v37", "v38", "v39", "v40", "v41", "v42", "v43", \
  "v44", "v45", "v46", "v47", "v48", "v49", "v50", "v51", "v52", "v53", "v54", "v55", \
  "v56", "v57", "v58", "v59", "v60", "v61", "v62", "v63", "v64", "v65", "v66", "v67", \
  "v68", "v69", "v70", "v71", "v72", "v73", "v74", "v75", "v76", "v77", "v78", "v79", \
  "v80", "v81", "v82", "v83", "v84", "v85", "v86", "v87", "v88", "v89", "v90", "v91", \
  "v92", "v93", "v94", "v95"
#define RW_CLOB_TOT \
  "v96", "v97", "v98", "v99", "v100", "v101", "v102", "v103", "v104", "v105", "v106", "v107", \
  "v108", "v109", "v110", "v111", "v112", "v113", "v114", "v115", "v116", "v117", "v118", "v119", \
  "v120", "v121", "v122", "v123", "v124", "v125", "v126", "v127", "v128", "v129", "v130", "v131", \
  "v132", "v133", "v134", "v135", "v136", "v137", "v138", "v139", "v140", "v141", "v142", "v143", \
  "v144", "v145", "v146", "v147", "v148", "v149", "v150", "v151", "v152", "v153", "v154", "v155", \
  "v156", "v157", "v158", "v159"
#define RW_CLOB_A \
  "v160", "v161", "v162", "v163", "v164", "v165", "v166", "v167", "v168", "v169", "v170", "v171", \
  "v172", "v173", "v174", "v175", "v176", "v177", "v178", "v179", "v180", "v181", "v182", "v183", \
  "v184", "v185", "v186", "v187", "v188", "v189", "v190", "v191", "v192", "v193", "v194", "v195", \
  "v196", "v197", "v198", "v199", "v200", "v201", "v202", "v203", "v204", "v205", "v206", "v207"
#define RW_CLOB_B \
  "v208", "v209", "v210", "v211", "v212", "v213", "v214", "v215", "v216", "v217", "v218", "v219", \
  "v220", "v221", "v222", "v223", "v224", "v225", "v226", "v227", "v228", "v229", "v230", "v231", \
  "v232", "v233", "v234", "v235", "v236", "v237", "v238", "v239", "v240", "v241", "v242", "v243", \
  "v244", "v245", "v246", "v247", "v248", "v249", "v250", "v251", "v252", "v253", "v254", "v255"
#define RW_ZERO \
  "v_mov_b32 v32, 0\n\t" "v_mov_b32 v33, 0\n\t" "v_mov_b32 v34, 0\n\t" "v_mov_b32 v35, 0\n\t" "v_mov_b32 v36, 0\n\t" "v_mov_b32 v37, 0\n\t" \
  "v_mov_b32 v38, 0\n\t" "v_mov_b32 v39, 0\n\t" "v_mov_b32 v40, 0\n\t" "v_mov_b32 v41, 0\n\t" "v_mov_b32 v42, 0\n\t" "v_mov_b32 v43, 0\n\t" \
  "v_mov_b32 v44, 0\n\t" "v_mov_b32 v45, 0\n\t" "v_mov_b32 v46, 0\n\t" "v_mov_b32 v47, 0\n\t" "v_mov_b32 v48, 0\n\t" "v_mov_b32 v49, 0\n\t" \
  "v_mov_b32 v50, 0\n\t" "v_mov_b32 v51, 0\n\t" "v_mov_b32 v52, 0\n\t" "v_mov_b32 v53, 0\n\t" "v_mov_b32 v54, 0\n\t" "v_mov_b32 v55, 0\n\t" \
  "v_mov_b32 v56, 0\n\t" "v_mov_b32 v57, 0\n\t" "v_mov_b32 v58, 0\n\t" "v_mov_b32 v59, 0\n\t" "v_mov_b32 v60, 0\n\t" "v_mov_b32 v61, 0\n\t" \
  "v_mov_b32 v62, 0\n\t" "v_mov_b32 v63, 0\n\t" "v_mov_b32 v64, 0\n\t" "v_mov_b32 v65, 0\n\t" "v_mov_b32 v66, 0\n\t" "v_mov_b32 v67, 0\n\t" \
  "v_mov_b32 v68, 0\n\t" "v_mov_b32 v69, 0\n\t" "v_mov_b32 v70, 0\n\t" "v_mov_b32 v71, 0\n\t" "v_mov_b32 v72, 0\n\t" "v_mov_b32 v73, 0\n\t" \
  "v_mov_b32 v74, 0\n\t" "v_mov_b32 v75, 0\n\t" "v_mov_b32 v76, 0\n\t" "v_mov_b32 v77, 0\n\t" "v_mov_b32 v78, 0\n\t" "v_mov_b32 v79, 0\n\t" \
  "v_mov_b32 v80, 0\n\t" "v_mov_b32 v81, 0\n\t" "v_mov_b32 v82, 0\n\t" "v_mov_b32 v83, 0\n\t" "v_mov_b32 v84, 0\n\t" "v_mov_b32 v85, 0\n\t" \
  "v_mov_b32 v86, 0\n\t" "v_mov_b32 v87, 0\n\t" "v_mov_b32 v88, 0\n\t" "v_mov_b32 v89, 0\n\t" "v_mov_b32 v90, 0\n\t" "v_mov_b32 v91, 0\n\t" \
  "v_mov_b32 v92, 0\n\t" "v_mov_b32 v93, 0\n\t" "v_mov_b32 v94, 0\n\t" "v_mov_b32 v95, 0\n\t" "v_mov_b32 v96, 0\n\t" "v_mov_b32 v97, 0\n\t" \
  "v_mov_b32 v98, 0\n\t" "v_mov_b32 v99, 0\n\t" "v_mov_b32 v100, 0\n\t" "v_mov_b32 v101, 0\n\t" "v_mov_b32 v102, 0\n\t" "v_mov_b32 v103, 0\n\t" \
  "v_mov_b32 v104, 0\n\t" "v_mov_b32 v105, 0\n\t" "v_mov_b32 v106, 0\n\t" "v_mov_b32 v107, 0\n\t" "v_mov_b32 v108, 0\n\t" "v_mov_b32 v109, 0\n\t" \
  "v_mov_b32 v110, 0\n\t" "v_mov_b32 v111, 0\n\t" "v_mov_b32 v112, 0\n\t" "v_mov_b32 v113, 0\n\t" "v_mov_b32 v114, 0\n\t" "v_mov_b32 v115, 0\n\t" \
  "v_mov_b32 v116, 0\n\t" "v_mov_b32 v117, 0\n\t" "v_mov_b32 v118, 0\n\t" "v_mov_b32 v119, 0\n\t" "v_mov_b32 v120, 0\n\t" "v_mov_b32 v121, 0\n\t" \
  "v_mov_b32 v122, 0\n\t" "v_mov_b32 v123, 0\n\t" "v_mov_b32 v124, 0\n\t" "v_mov_b32 v125, 0\n\t" "v_mov_b32 v126, 0\n\t" "v_mov_b32 v127, 0\n\t" \
  "v_mov_b32 v128, 0\n\t" "v_mov_b32 v129, 0\n\t" "v_mov_b32 v130, 0\n\t" "v_mov_b32 v131, 0\n\t" "v_mov_b32 v132, 0\n\t" "v_mov_b32 v133, 0\n\t" \
  "v_mov_b32 v134, 0\n\t" "v_mov_b32 v135, 0\n\t" "v_mov_b32 v136, 0\n\t" "v_mov_b32 v137, 0\n\t" "v_mov_b32 v138, 0\n\t" "v_mov_b32 v139, 0\n\t" \
  "v_mov_b32 v140, 0\n\t" "v_mov_b32 v141, 0\n\t" "v_mov_b32 v142, 0\n\t" "v_mov_b32 v143, 0\n\t" "v_mov_b32 v144, 0\n\t" "v_mov_b32 v145, 0\n\t" \
  "v_mov_b32 v146, 0\n\t" "v_mov_b32 v147, 0\n\t" "v_mov_b32 v148, 0\n\t" "v_mov_b32 v149, 0\n\t" "v_mov_b32 v150, 0\n\t" "v_mov_b32 v151, 0\n\t" \
  "v_mov_b32 v152, 0\n\t" "v_mov_b32 v153, 0\n\t" "v_mov_b32 v154, 0\n\t" "v_mov_b32 v155, 0\n\t" "v_mov_b32 v156, 0\n\t" "v_mov_b32 v157, 0\n\t" \
  "v_mov_b32 v158, 0\n\t" "v_mov_b32 v159, 0\n\t"

__device__ __forceinline__ void rw_zero() { asm volatile(RW_ZERO ::: RW_CLOB_SUB, RW_CLOB_TOT); }

// Running sums += block sums, block sums = 0 (plain VALU, outside index mode).
__device__ __forceinline__ void rw_fold() {
  asm volatile(RW_FOLDG0 RW_FOLDG1 RW_FOLDG2 RW_FOLDG3 ::: RW_CLOB_SUB, RW_CLOB_TOT);
}

// Waits for every LDS read in flight (the window about to be added).
__device__ __forceinline__ void rw_wait() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// Waits for the LDS reads in flight, then issues the reads of a window into buffer BUF
// (0: A, 1: B): n chunks (2 <= n <= 12, the chunks this wavefront's trials touch in this
// channel); `addr` is this lane's window start in LDS.
#define RW_MORE(i, lo, hi, off) \
  "s_cmp_lt_u32 %[n], " #i "\n\ts_cbranch_scc1 1f\n\t" RW_LD(lo, hi, off)
template <int BUF>
__device__ __forceinline__ void rw_load(unsigned addr, int n) {
  if constexpr (BUF == 0)
    asm volatile("s_waitcnt lgkmcnt(0)\n\t" RW_LD(160, 163, 0) RW_LD(164, 167, 16)
                 RW_MORE(3, 168, 171, 48) RW_MORE(4, 172, 175, 64) RW_MORE(5, 176, 179, 96)
                 RW_MORE(6, 180, 183, 112) RW_MORE(7, 184, 187, 144) RW_MORE(8, 188, 191, 160)
                 RW_MORE(9, 192, 195, 192) RW_MORE(10, 196, 199, 208) RW_MORE(11, 200, 203, 240)
                 RW_MORE(12, 204, 207, 256) "1:"
                 : : [na] "v"(addr), [n] "s"(n) : "memory", "scc", RW_CLOB_A);
  else
    asm volatile("s_waitcnt lgkmcnt(0)\n\t" RW_LD(208, 211, 0) RW_LD(212, 215, 16)
                 RW_MORE(3, 216, 219, 48) RW_MORE(4, 220, 223, 64) RW_MORE(5, 224, 227, 96)
                 RW_MORE(6, 228, 231, 112) RW_MORE(7, 232, 235, 144) RW_MORE(8, 236, 239, 160)
                 RW_MORE(9, 240, 243, 192) RW_MORE(10, 244, 247, 208) RW_MORE(11, 248, 251, 240)
                 RW_MORE(12, 252, 255, 256) "1:"
                 : : [na] "v"(addr), [n] "s"(n) : "memory", "scc", RW_CLOB_B);
}

// The eight trials of one channel from window BUF: trial g adds window registers
// idx_g .. idx_g + 7 (index byte g of i0:i1) into its block sums.
template <int BUF>
__device__ __forceinline__ void rw_trials(int i0, int i1) {
  int t;
  if constexpr (BUF == 0)
    asm volatile(RW_IDX_ON(i0, RW_B0) RW_TA0 RW_IDX(i0, RW_B1) RW_TA1 RW_IDX(i0, RW_B2) RW_TA2 RW_IDX(i0, RW_B3) RW_TA3
                 RW_IDX(i1, RW_B0) RW_TA4 RW_IDX(i1, RW_B1) RW_TA5 RW_IDX(i1, RW_B2) RW_TA6 RW_IDX(i1, RW_B3) RW_TA7
                 "s_set_gpr_idx_off"
                 : [t] "=&s"(t)
                 : [i0] "s"(i0), [i1] "s"(i1)
                 : "m0", "scc", RW_CLOB_SUB);
  else
    asm volatile(RW_IDX_ON(i0, RW_B0) RW_TB0 RW_IDX(i0, RW_B1) RW_TB1 RW_IDX(i0, RW_B2) RW_TB2 RW_IDX(i0, RW_B3) RW_TB3
                 RW_IDX(i1, RW_B0) RW_TB4 RW_IDX(i1, RW_B1) RW_TB5 RW_IDX(i1, RW_B2) RW_TB6 RW_IDX(i1, RW_B3) RW_TB7
                 "s_set_gpr_idx_off"
                 : [t] "=&s"(t)
                 : [i0] "s"(i0), [i1] "s"(i1)
                 : "m0", "scc", RW_CLOB_SUB);
}

// Running sums of trial G into compiler registers.
template <int G>
__device__ __forceinline__ void rw_get(float (&x)[8]) {
#define RW_GET_CASE(g) \
  if constexpr (G == g) \
    asm volatile(RW_GET##g : "=v"(x[0]), "=v"(x[1]), "=v"(x[2]), "=v"(x[3]), "=v"(x[4]), "=v"(x[5]), "=v"(x[6]), "=v"(x[7]));
  RW_GET_CASE(0) RW_GET_CASE(1) RW_GET_CASE(2) RW_GET_CASE(3) RW_GET_CASE(4) RW_GET_CASE(5) RW_GET_CASE(6)
  RW_GET_CASE(7)
#undef RW_GET_CASE
}

// The eight records {window byte offset, trial indices 0-3, 4-7, 0} of a stage's channels
// for this wavefront (records 128 bytes apart), by scalar loads waited for at once. Issued
// at a stage start, where no LDS read is in flight, so the wait costs one scalar-cache
// latency per stage. The table carries seven padding channels, so the last stage's reads
// stay inside it. The outputs are early-clobber: a load whose destination overlapped the
// base address would overwrite it while later loads of the group still read it.
__device__ __forceinline__ void load_stage_meta(const int4* base, int4 (&m)[kRwCs]) {
  asm volatile(
      "s_load_dwordx4 %0, %8, 0x0\n\t"
      "s_load_dwordx4 %1, %8, 0x80\n\t"
      "s_load_dwordx4 %2, %8, 0x100\n\t"
      "s_load_dwordx4 %3, %8, 0x180\n\t"
      "s_load_dwordx4 %4, %8, 0x200\n\t"
      "s_load_dwordx4 %5, %8, 0x280\n\t"
      "s_load_dwordx4 %6, %8, 0x300\n\t"
      "s_load_dwordx4 %7, %8, 0x380\n\t"
      "s_waitcnt lgkmcnt(0)"
      : "=&s"(m[0]), "=&s"(m[1]), "=&s"(m[2]), "=&s"(m[3]), "=&s"(m[4]), "=&s"(m[5]), "=&s"(m[6]), "=&s"(m[7])
      : "s"(base)
      : "memory");
}

// Wavefront w's DMAs for stage sd: channel sd * 8 + w (clamped to the last channel, which
// keeps the per-wavefront DMA count uniform). Slot position m (16 bytes) holds samples
// 8q + 4r .. + 3 for m = 3q + r, r < 2; r = 2 is padding (filled with the r = 1 samples).
template <bool RING>
__device__ __forceinline__ void rw_stage_dma(const RWParams& P, unsigned sbase, int sd, int w, int64_t t0, int grp,
                                             int lane, int w0) {
  int c = sd * kRwCs + w;
  if (c >= P.nchan) c = P.nchan - 1;
  const dd::ci32_t gb = (dd::ci32_t)(P.gbase + (int64_t)grp * P.nchan);
  const int first = (int)t0 + gb[c];
  int start = first;
  if constexpr (RING) {
    start += w0;
    if (start >= (int)P.in.ring_len) start -= (int)P.in.ring_len;
  }
  const char* rp = static_cast<const char*>(P.in.ptr) + (int64_t)c * P.in.row_stride * 4;
  const unsigned slot = sbase + (unsigned)((sd % P.nb) * kRwCs + w) * 1024u * (unsigned)P.ndma;
  if (RING || first + P.xs <= (int)P.in.nvalid) {
    for (int j = 0; j < P.ndma; ++j) {
      const int m = 64 * j + lane;
      const int q = m / 3, r = m - 3 * q;
      dd::dma_x4(rp, 4u * (unsigned)(start + 8 * q + 4 * min(r, 1)), slot + 1024u * (unsigned)j);
    }
  } else {
    // the data ends inside this slot: one 4-byte DMA per sample, each clamped to the last
    // sample, then wait for them so the vmcnt bookkeeping of later stages stays exact
    const int nlim = (int)P.in.nvalid - 1;
    for (int j = 0; j < P.ndma; ++j)
      for (int k = 0; k < 4; ++k) {
        const int m = 64 * j + 16 * k + (lane >> 2);
        const int q = m / 3, r = m - 3 * q;
        const int pos = first + 8 * q + 4 * min(r, 1) + (lane & 3);
        dd::dma<4>(rp, 4u * (unsigned)min(pos, nlim), slot + 1024u * (unsigned)j + 256u * (unsigned)k);
      }
    dd::wait_vm(0);
  }
}

// Trial G's outputs (float4 stores when aligned) and FP64 statistics partials.
template <int G>
__device__ __forceinline__ void rw_store(const RWParams& P, int dw, int64_t t0, int64_t tile, int lane, bool vec_ok) {
  float x[8];
  rw_get<G>(x);
  const int d = dw + G;
  if (d >= P.ndm) return;
  float* orow = P.out + (int64_t)d * P.out_stride;
  const int64_t tb = t0 + 8 * lane;
  if (vec_ok && tb + 7 < P.nout) {
    *reinterpret_cast<float4*>(orow + tb) = make_float4(x[0], x[1], x[2], x[3]);
    *reinterpret_cast<float4*>(orow + tb + 4) = make_float4(x[4], x[5], x[6], x[7]);
  } else {
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (tb + j < P.nout) orow[tb + j] = x[j];
  }
  if (P.part) {
    double s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (tb + j < P.nout) {
        const double v = x[j];
        s1 += v;
        s2 += v * v;
      }
    }
    s1 = dd::wave_sum_fixed(s1);
    s2 = dd::wave_sum_fixed(s2);
    if (lane == 0) {
      const int64_t nseg = (P.nout + 511) / 512;
      P.part[((int64_t)d * nseg + tile) * 2] = s1;
      P.part[((int64_t)d * nseg + tile) * 2 + 1] = s2;
    }
  }
}

// One work unit per workgroup; each XCD (workgroups lin, lin + 8, ...) takes a contiguous
// run of units, tile-major, so the DM groups of a tile share that XCD's L2.
template <bool RING>
__global__ __launch_bounds__(512) __attribute__((amdgpu_num_vgpr(16))) void dedisp_regwin(RWParams P) {
  extern __shared__ __align__(16) float smem[];
  const int64_t lin = blockIdx.x;
  const int64_t per = (P.nitems + 7) / 8;
  const int64_t item = (lin & 7) * per + (lin >> 3);
  if (item >= P.nitems) return;  // uniform for the workgroup, before any barrier
  const int64_t tile = item / P.ngroups;
  const int grp = (int)(item - tile * P.ngroups);
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t t0 = tile * 512;
  const unsigned sbase = dd::lds_addr(smem);
  const unsigned slot_bytes = 1024u * (unsigned)P.ndma;
  const unsigned stage_bytes = (unsigned)kRwCs * slot_bytes;
  const int w0 = RING ? (int)(P.in.win0 % P.in.ring_len) : 0;
  rw_zero();
  const int pre = min(P.nb - 1, P.nstages);
  for (int sd = 0; sd < pre; ++sd) rw_stage_dma<RING>(P, sbase, sd, w, t0, grp, lane, w0);
  const int4* mg = P.meta + (int64_t)grp * P.nchan * kRwWaves + w;  // channel c: mg[8c]
  const unsigned lane48 = 48u * (unsigned)lane;                      // 12 words per 8 samples
  for (int st = 0; st < P.nstages; ++st) {
    // stages issued after st: min(nstages - 1, st + nb - 2) - st
    const int later = min(P.nstages - 1, st + P.nb - 2) - st;
    dd::wait_vm(later * P.ndma);
    dd::block_barrier();
    const int c0 = st * kRwCs;
    if ((c0 & (DD_CHAN_BLOCK - 1)) == 0 && c0 != 0) rw_fold();
    const int n_here = min(kRwCs, P.nchan - c0);
    const unsigned slot0 = sbase + (unsigned)(st % P.nb) * stage_bytes + lane48;
    int4 mt[kRwCs];
    load_stage_meta(mg + (int64_t)c0 * kRwWaves, mt);
    rw_load<0>(slot0 + (unsigned)mt[0].x, mt[0].w);
#pragma unroll
    for (int cc = 0; cc < kRwCs; ++cc) {
      if (cc >= n_here) break;
      const bool nxt = cc + 1 < n_here;
      const unsigned na = slot0 + (unsigned)(cc + 1) * slot_bytes + (unsigned)mt[cc + 1 < kRwCs ? cc + 1 : cc].x;
      if (cc & 1) {
        if (nxt)
          rw_load<0>(na, mt[cc + 1 < kRwCs ? cc + 1 : cc].w);
        else
          rw_wait();
        rw_trials<1>(mt[cc].y, mt[cc].z);
      } else {
        if (nxt)
          rw_load<1>(na, mt[cc + 1 < kRwCs ? cc + 1 : cc].w);
        else
          rw_wait();
        rw_trials<0>(mt[cc].y, mt[cc].z);
      }
      // the next ring stage's DMAs go out after this stage's first channel, not in a burst
      // of every wavefront right after the barrier
      if (cc == 0 && st + P.nb - 1 < P.nstages) rw_stage_dma<RING>(P, sbase, st + P.nb - 1, w, t0, grp, lane, w0);
    }
  }
  rw_fold();

  const bool vec_ok = ((P.out_stride & 3) == 0) && ((reinterpret_cast<uintptr_t>(P.out) & 15) == 0);
  const int dw = grp * (kRwWaves * kRwG) + w * kRwG;
  rw_store<0>(P, dw, t0, tile, lane, vec_ok);
  rw_store<1>(P, dw, t0, tile, lane, vec_ok);
  rw_store<2>(P, dw, t0, tile, lane, vec_ok);
  rw_store<3>(P, dw, t0, tile, lane, vec_ok);
  rw_store<4>(P, dw, t0, tile, lane, vec_ok);
  rw_store<5>(P, dw, t0, tile, lane, vec_ok);
  rw_store<6>(P, dw, t0, tile, lane, vec_ok);
  rw_store<7>(P, dw, t0, tile, lane, vec_ok);
}

using RwFn = void (*)(RWParams);

}  // namespace

namespace dd {

int launch_regwin(const dd_plan* p, const InView& in, const int32_t* d_table, int64_t nout, float* out,
                  int64_t out_stride, double* part, void* stream) {
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Launch& g = p->launch;
  if (in.nvalid >= (int64_t)1 << 30 || in.ring_len >= (int64_t)1 << 30)
    return fail(DD_ERR_UNSUPPORTED, "windows of 2^30 samples or more per channel are not supported");
  const int64_t ntiles = (nout + kTile - 1) / kTile;
  RWParams P{};
  P.in = in;
  P.gbase = d_table;
  P.meta = reinterpret_cast<const int4*>(d_table + rw_meta_offset(p));
  P.out = out;
  P.part = part;
  P.out_stride = out_stride;
  P.nout = nout;
  P.nitems = ntiles * p->ngroups;
  P.nchan = p->nchan;
  P.ndm = p->ndm;
  P.ngroups = p->ngroups;
  P.xs = g.L;
  P.ndma = g.nd;
  P.nb = g.nb;
  P.nstages = (p->nchan + kRwCs - 1) / kRwCs;
  RwFn k = in.ring_len > 0 ? dedisp_regwin<true> : dedisp_regwin<false>;
  if (g.lds > 65536) {
    hipError_t e = hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)g.lds);
    if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
  }
  const int64_t nblocks = (P.nitems + 7) / 8 * 8;
  if (nblocks > 0x7fffffff) return fail(DD_ERR_UNSUPPORTED, "too many work items");
  if (nblocks == 0) return DD_OK;
  hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(64 * kRwWaves), (size_t)g.lds, st, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(DD_ERR_HIP, std::string("dedisp_regwin launch: ") + hipGetErrorString(e));
  return DD_OK;
}

}  // namespace dd
