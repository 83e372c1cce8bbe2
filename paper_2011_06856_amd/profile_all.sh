#!/bin/bash
# rocprofv3 summaries of the two step kernels on their benchmark workloads:
#   k_stream_collide  circular shock 1024^2, 256 velocities, FP32 (tile kernel)
#   k_push_step       quadrant problem 2048^2, 1536 velocities, order 5, FP32 and
#                     bfloat16 deviations (push kernel)
# Per workload: a kernel-trace/stats run, then a FETCH_SIZE run and a WRITE_SIZE
# run (counters in passes of their own), each ending with a 1 GiB device copy
# that calibrates the counters to bytes.  Run from the repository root on a
# GPU machine:  bash paper_2011_06856_amd/profile_all.sh OUT_DIR
# Writes OUT_DIR/raw/... (rocprofv3 CSV) and OUT_DIR/<name>.md/.json.
set -e
OUT=${1:-profile_out}
export TMPDIR=/tmp
SQ1="SQ_WAVES SQ_INSTS_VALU SQ_INSTS_MFMA SQ_INSTS_VMEM_RD SQ_INSTS_SMEM SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES"
SQ2="SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_ANY SQ_VALU_MFMA_BUSY_CYCLES SQ_INSTS_VMEM_WR SQ_WAIT_ANY SQ_INSTS_LDS SQ_ACTIVE_INST_SCA"
run() {   # name, kernel, launch bytes, wave-velocities per launch, stats args, counter args
    local name=$1 kernel=$2 bytes=$3 units=$4 sargs=$5 cargs=$6
    local D=$OUT/raw/$name
    timeout -s KILL 180 rocprofv3 --kernel-trace --stats -d $D/stats -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run $sargs
    timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d $D/fetch -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run $cargs
    timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d $D/write -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run $cargs
    timeout -s KILL 120 rocprofv3 --pmc $SQ1 -d $D/sq1 -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run $cargs
    timeout -s KILL 120 rocprofv3 --pmc $SQ2 -d $D/sq2 -o run --output-format csv -- \
        python3 -m paper_2011_06856_amd.profile_run $cargs
    python3 -m paper_2011_06856_amd.profile_summary --stats $D/stats --fetch $D/fetch --write $D/write \
        --sq $D/sq1 $D/sq2 --wave-units $units \
        --name $name --kernel "$kernel" --launch-bytes $bytes --out-dir $OUT \
        --command "rocprofv3 --kernel-trace --stats -- python3 -m paper_2011_06856_amd.profile_run $sargs ; rocprofv3 --pmc FETCH_SIZE -- python3 -m paper_2011_06856_amd.profile_run $cargs ; rocprofv3 --pmc WRITE_SIZE -- python3 -m paper_2011_06856_amd.profile_run $cargs ; rocprofv3 --pmc $SQ1 -- (same) ; rocprofv3 --pmc $SQ2 -- (same) (bash paper_2011_06856_amd/profile_all.sh)"
}
# algorithmic bytes per launch: 8 B per site-velocity (FP32 read + write);
# wave-velocities: site-velocity updates / 64
run stream_collide_f32_circular_1024 "k_stream_collide<float, float, 3, 64, false>" 2147483648 4194304 \
    "--steps 200" "--steps 4"
run push_step_f32_quadrant_2048 "k_push_step<float, float, 5, 8, false, false>" 51539607552 100663296 \
    "--workload quadrant --side 2048 --steps 20" "--workload quadrant --side 2048 --steps 3"
# bfloat16 deviations: 4 B per site-velocity plus the per-site equilibrium
# coefficients (6 shells x 11 FP32, read and written: 528 B per site)
run push_step_bf16dev_quadrant_2048 "k_push_step<float, unsigned short, 5, 8, false, true>" 27980857344 100663296 \
    "--workload quadrant --side 2048 --steps 20 --precision bf16dev" \
    "--workload quadrant --side 2048 --steps 3 --precision bf16dev"

# The 48-problem batch (FP32, the library's default work-group shape and
# mode, one graph replay per step): kernel statistics only, with the kernel
# time of one step summed over the launches a step makes.
D=$OUT/raw/batch48
mkdir -p $D
SV=$(python3 -c "import workloads as W; print(sum(p['Np'] * p['K'] * p['nx'] * p['ny'] for p in W.batch_problems(48, seed=0, steps=1)))")
timeout -s KILL 180 rocprofv3 --kernel-trace --stats -d $D/stats -o run --output-format csv -- \
    python3 -m paper_2011_06856_amd.profile_run --workload batch48 --steps 40 > $D.out.txt
python3 -m paper_2011_06856_amd.profile_summary --stats $D/stats --name batch_step_f32_batch48 \
    --kernel k_batch_step --launch-bytes 0 --out-dir $OUT \
    --step-kernels k_batch_step,k_batch_flat,k_push_batch --steps 40 --sv-per-step $SV \
    --command "rocprofv3 --kernel-trace --stats -- python3 -m paper_2011_06856_amd.profile_run --workload batch48 --steps 40 (bash paper_2011_06856_amd/profile_all.sh)"
{ echo; echo "Program output: \`$(grep profile_run: $D.out.txt)\`"; } >> $OUT/batch_step_f32_batch48.md

# The learned form's readout network (FP32 matrix cores): kernel statistics and
# one pass of SQ counters, summarised for the fused inference kernel and for
# the training GEMM.
D=$OUT/raw/mlp
MLPSQ="SQ_WAVES SQ_INSTS_VALU SQ_INSTS_MFMA SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CYCLES SQ_WAVE_CYCLES SQ_ACTIVE_INST_VALU SQ_ACTIVE_INST_ANY"
mkdir -p $D
timeout -s KILL 180 rocprofv3 --kernel-trace --stats -d $D/stats -o run --output-format csv -- \
    python3 -m paper_2011_06856_amd.profile_run --workload mlp --side 512 --steps 20 > $D.out.txt
timeout -s KILL 120 rocprofv3 --pmc $MLPSQ -d $D/sq -o run --output-format csv -- \
    python3 -m paper_2011_06856_amd.profile_run --workload mlp --side 512 --steps 5
for k in k_mlp_fused k_gemm_mfma; do
    python3 -m paper_2011_06856_amd.profile_summary --stats $D/stats --sq $D/sq --name mlp_${k#k_}_512 \
        --kernel $k --launch-bytes 0 --out-dir $OUT \
        --command "rocprofv3 --kernel-trace --stats -- python3 -m paper_2011_06856_amd.profile_run --workload mlp --side 512 --steps 20 ; rocprofv3 --pmc $MLPSQ -- python3 -m paper_2011_06856_amd.profile_run --workload mlp --side 512 --steps 5 (bash paper_2011_06856_amd/profile_all.sh)"
    { echo; echo "Program output: \`$(grep profile_run: $D.out.txt)\`"; } >> $OUT/mlp_${k#k_}_512.md
done
